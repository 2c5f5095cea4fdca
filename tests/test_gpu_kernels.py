"""GPU parity of the kernel-level pieces against the FP64 oracle, called through the C-ABI:
Philox draws (bit-exact), MLS shape functions, and the stochastic bond update (bit-exact
over more than a million element-steps)."""
import sys

import numpy as np
import pytest

from paper_1808_01448_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1808_01448_amd import lbib

    lbib.lib()
    return lbib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_philox_bit_exact(L, orc):
    n = 1 << 20
    ctr = W.random_u32(1, (n, 4))
    key = W.random_u32(2, (n, 2))
    ctr[:3] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]]
    key[:3] = [[0, 0], [0xFFFFFFFF] * 2, [0xA4093822, 0x299F31D0]]
    say("philox: n =", n)
    out = L.philox(_dev(ctr.view(np.int32)), _dev(key.view(np.int32)))
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    ref = orc.philox_batch(ctr, key)
    np.testing.assert_array_equal(got, ref)
    assert got[0].tolist() == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


@pytest.mark.parametrize("nx,ny", [(40, 24), (257, 33), (4096, 1024)])
def test_mls_matches_oracle(L, orc, nx, ny):
    pts = W.random_points(5, 6000, nx, ny)
    say("mls:", nx, ny, len(pts))
    node, phi, psx, psy = L.mls(_dev(pts), nx, ny)
    torch.cuda.synchronize()
    node, phi, psx, psy = (t.cpu().numpy() for t in (node, phi, psx, psy))
    for k, (x, y) in enumerate(pts):
        r = orc.mls(nx, ny, x, y)
        ni, nj, rphi, rpsx, rpsy = r
        sel = node[k, :, 0] >= 0
        got = sorted(zip(node[k, sel, 1], node[k, sel, 0], phi[k, sel], psx[k, sel], psy[k, sel]))
        ref = sorted(zip(nj, ni, rphi, rpsx, rpsy))
        assert [(a, b) for a, b, *_ in got] == [(a, b) for a, b, *_ in ref], (x, y)
        # two different 3x3 solvers (cofactors here, pivoted elimination in the oracle); the
        # wall-cut supports have condition numbers up to ~1e5
        np.testing.assert_allclose([g[2] for g in got], [r_[2] for r_ in ref], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose([g[3] for g in got], [r_[3] for r_ in ref], rtol=1e-10, atol=1e-11)
        np.testing.assert_allclose([g[4] for g in got], [r_[4] for r_ in ref], rtol=1e-10, atol=1e-11)


def test_bonds_bit_exact(L, orc):
    """4096 independent particles x 256 elements = 1 048 576 element-steps, with mixed
    ligands, distances straddling y_cr and pre-existing bonds."""
    sets, nl = 4096, 256
    g = np.random.default_rng(9)
    ligand = (g.random((sets, nl)) < 0.7).astype(np.uint8)
    d = g.uniform(0.0, 1.2, (sets, nl))
    b_in = ((g.random((sets, nl)) < 0.3) & (ligand == 1)).astype(np.uint8)
    step = g.integers(0, 2**40, sets).astype(np.int64)
    params = dict(y_cr=0.6, y_eq=0.3, sigma=3.0, sigma_star=1.5, k_f=0.9, k_r0=0.02, kBT=0.05)
    seed = 0x123456789ABCDEF
    say("bonds:", sets, "x", nl)
    b_out, nb, npr = L.bonds(_dev(ligand), _dev(d), _dev(b_in), _dev(step), tuple(params.values()), seed, pid=3)
    torch.cuda.synchronize()
    b_out, nb, npr = b_out.cpu().numpy(), nb.cpu().numpy(), npr.cpu().numpy()
    for s in range(sets):
        ref, rnb, rnp = orc.bonds(ligand[s], d[s], b_in[s], **params, seed=seed, step=int(step[s]), pid=3)
        np.testing.assert_array_equal(b_out[s], ref)
        assert nb[s] == rnb and npr[s] == rnp
    # both transitions are exercised
    assert ((b_in == 1) & (b_out == 0)).sum() > 1000 and ((b_in == 0) & (b_out == 1)).sum() > 1000


def test_bandwidth_probe_runs(L):
    v = L.bandwidth_probe(1 << 28, 3)
    say("copy GB/s", v)
    assert v > 100.0
