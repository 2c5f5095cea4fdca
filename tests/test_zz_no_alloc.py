"""The allocation-free solve (lbib_solve_static) against the handle-based calls it replaces
(lbib_create ... lbib_step with the serial schedule): the per-step particle records and the
final bond flags must be bit-identical.  Two solves in a row, the second on a smaller
lattice with a smaller particle, so the second runs on the static array the first left
behind.  Through the C-ABI, on the GPU."""
import numpy as np
import pytest

from paper_1808_01448_amd import lbib
from paper_1808_01448_amd import workloads as W

pytestmark = pytest.mark.gpu


def _handle_run(w, n):
    s = lbib.Sim(w)
    s.set_overlap(0)
    s.trace_enable(n)
    s.step(n)
    s.sync()
    tr = s.trace(n)
    b, _ = s.bonds()
    s.close()
    return tr, b


def _cases():
    big = W.channel_small_binding("fp64")
    big["lattice"].update(nx=160, ny=64)
    big["particle"].update(xc=50.0)
    small = W.channel_small_binding("fp32")
    small["lattice"].update(nx=72, ny=40)
    small["particle"].update(xc=30.0, a_major=5.0, b_minor=5.0, n_markers=40)
    small["particle"]["yc"] = -0.5 + 0.5 * W.Y_CR_HAT * 40 + 5.0
    return [("fp64_160x64_r8", big, 300), ("fp32_72x40_r5", small, 200)]


def test_static_solve_matches_the_handle_path_twice():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    for name, w, n in _cases():
        print(f"static solve {name}, {n} steps", flush=True)
        tr_s, b_s = lbib.solve_static(w, n)
        tr_h, b_h = _handle_run(w, n)
        assert tr_s.shape == tr_h.shape == (n, len(lbib.STATE_FIELDS))
        np.testing.assert_array_equal(tr_s.view(np.uint64), tr_h.view(np.uint64), err_msg=name)
        np.testing.assert_array_equal(b_s, b_h, err_msg=name)
        assert tr_h[:, lbib.STATE_FIELDS.index("n_bonds")].max() > 0, name  # bonds formed


def test_static_solve_refuses_a_particle_beyond_the_static_area():
    w = W.channel_small_fp64()
    w["lattice"].update(nx=1024, ny=1024)
    w["particle"].update(a_major=200.0, b_minor=200.0, xc=512.0, yc=220.0, n_markers=1024)
    with pytest.raises(lbib.LbibError) as e:
        lbib.solve_static_bytes(w)
    assert e.value.status == lbib.E_INVALID and "static area" in str(e.value)


def test_static_solve_reports_the_population_bytes():
    w = W.channel_small_fp64()
    need = lbib.solve_static_bytes(w)
    assert need >= 2 * 9 * 8 * w["lattice"]["nx"] * w["lattice"]["ny"]
    assert need % 256 == 0
