// lbib_host.cpp -- host pieces shared by the single-simulation handle and the pool.
#include "lbib_host.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace lbib {

namespace {

constexpr double kWq[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                           1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
constexpr int kExq[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEyq[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOppq[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Ligand-bearing elements: with rho_l = p/q in lowest terms, element l carries a ligand when
// floor((l+1) p/q) - floor(l p/q) = 1 -- floor(nl p/q) ligands spread evenly.
std::vector<uint8_t> ligand_layout(int nl, int p, int q)
{
    const int g = std::gcd(p, q);
    p /= g;
    q /= g;
    std::vector<uint8_t> out(nl);
    for (int l = 0; l < nl; ++l) out[l] = (uint8_t)((((int64_t)(l + 1) * p) / q - ((int64_t)l * p) / q) == 1);
    return out;
}

}  // namespace

uint16_t f32_to_f16(float f)
{
    uint32_t x;
    std::memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u, ax = x & 0x7fffffffu;
    if (ax >= 0x7f800000u) return (uint16_t)(sign | (ax > 0x7f800000u ? 0x7e00u : 0x7c00u));
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // rounds to infinity (>= 65520)
    if (ax < 0x33000000u) return (uint16_t)sign;                 // below 2^-25: rounds to zero
    const int e = (int)(ax >> 23) - 127 + 15;
    uint32_t m = ax & 0x7fffffu;
    if (e <= 0) {  // subnormal result: m_h = M 2^(e - 14), M the 24-bit significand
        m |= 0x800000u;
        const int shift = 14 - e;
        uint32_t r = m >> shift;
        const uint32_t rem = m & ((1u << shift) - 1u), halfway = 1u << (shift - 1);
        if (rem > halfway || (rem == halfway && (r & 1u))) ++r;
        return (uint16_t)(sign | r);
    }
    uint32_t r = ((uint32_t)e << 10) | (m >> 13);
    const uint32_t rem = m & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (r & 1u))) ++r;  // a carry moves into the exponent
    return (uint16_t)(sign | r);
}

float f16_to_f32(uint16_t h)
{
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16, e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    uint32_t x;
    if (e == 0) {
        const float v = std::ldexp((float)m, -24);  // zero or subnormal, exact
        return sign ? -v : v;
    }
    if (e == 31)
        x = sign | 0x7f800000u | (m << 13);
    else
        x = sign | ((e + 112u) << 23) | (m << 13);
    float f;
    std::memcpy(&f, &x, 4);
    return f;
}

uint16_t f32_to_bf16(float f)
{
    uint32_t x;
    std::memcpy(&x, &f, 4);
    x = (x & 0x7fffffffu) > 0x7f800000u ? 0x7fc00000u : x + 0x7fffu + ((x >> 16) & 1u);
    return (uint16_t)(x >> 16);
}

float bf16_to_f32(uint16_t h)
{
    const uint32_t x = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &x, 4);
    return f;
}

int64_t host_pop_index(const LatticeGeom& g, int q, int i, int j)
{
    if (g.pull) {
        const int sj = j - kEyq[q];
        if (sj < 0 || sj >= g.ny) return kOppq[q] * g.plane + (int64_t)j * g.pitch + i;
        int si = i - kExq[q];
        si = si < 0 ? si + g.nx : (si >= g.nx ? si - g.nx : si);
        return q * g.plane + (int64_t)sj * g.pitch + si;
    }
    return q * g.plane + (int64_t)j * g.pitch + i;
}

lbib_status check_lattice(const lbib_lattice_desc& d, std::string& msg)
{
    if (d.nx < 4 || d.ny < 4) return msg = "nx and ny must be >= 4", LBIB_E_INVALID;
    if ((int64_t)d.nx * d.ny > (int64_t)1 << 31) return msg = "more than 2^31 nodes", LBIB_E_INVALID;
    if (!is_finite(d.tau) || !(d.tau > 0.5)) return msg = "tau must be > 1/2", LBIB_E_INVALID;
    if (!is_finite(d.re) || d.re < 0) return msg = "Re must be >= 0", LBIB_E_INVALID;
    if (d.drive != 0 && d.drive != 1) return msg = "drive must be 0 (Poiseuille) or 1 (moving top wall)", LBIB_E_INVALID;
    if (d.precision < LBIB_FP64 || d.precision > LBIB_BF16_NEQ)
        return msg = "precision must be one of LBIB_FP64, LBIB_FP32, LBIB_FP16, LBIB_BF16, LBIB_FP16_NEQ, LBIB_BF16_NEQ",
               LBIB_E_UNSUPPORTED;
    return LBIB_OK;
}

LatticeGeom lattice_geom(const lbib_lattice_desc& d)
{
    LatticeGeom g;
    g.nx = d.nx;
    g.ny = d.ny;
    g.precision = d.precision;
    g.elem = d.precision == LBIB_FP64 ? 8 : d.precision == LBIB_FP32 ? 4 : 2;
    g.neq = d.precision == LBIB_FP16_NEQ || d.precision == LBIB_BF16_NEQ;
    const int align = (int)(256 / g.elem);  // rows start on 256-byte boundaries
    const int row = (d.nx + align - 1) / align * align;
    if (9 * (int64_t)row > INT32_MAX) {
        // population planes [q][j][i] (the pitch is a 32-bit value); the f - f_eq storages'
        // three moment planes follow
        g.pitch = row;
        g.plane = (int64_t)row * d.ny;
        g.mpitch = row;
    } else {
        // row-interleaved [j][q][i]: the nine population segments of a row are adjacent, so
        // a tile's eighteen access streams fall into a few DRAM pages instead of eighteen
        // planes a buffer apart; the f - f_eq storages' moments follow as rows [j][k][i]
        g.pitch = 9 * row;
        g.plane = row;
        g.mpitch = 3 * row;
        g.interleaved = true;
    }
    g.row = row;
    const double H = (double)d.ny;
    g.tau = d.tau;
    g.nu = (d.tau - 0.5) / 3.0;
    g.umax = d.re * g.nu / H;
    g.drive = d.drive;
    g.gx = d.drive == 1 ? 0.0 : 8.0 * g.nu * g.umax / (H * H);
    g.gy = 0.0;
    g.uw = d.drive == 1 ? g.umax : 0.0;
    g.buf_bytes = (size_t)9 * g.row * d.ny * g.elem + (g.neq ? (size_t)3 * g.row * d.ny * 4 : 0);
    g.upd_bytes = (int)(18 * g.elem) + (g.neq ? 24 : 0);
    if (d.precision == LBIB_FP16 || d.precision == LBIB_FP16_NEQ) {
        // the largest deviation f - w to expect is that of the rest population at a few times
        // u_max; a power of two maps it to ~2^13, far below the binary16 maximum (65504) and
        // far above its subnormal range (< 2^-14)
        const double u = std::max(4.0 * g.umax, 1e-6);
        const double dev = (4.0 / 9.0) * (3.0 * u + 4.5 * u * u);
        g.scale = std::ldexp(1.0, std::min(40, std::max(0, (int)std::floor(std::log2(8192.0 / dev)))));
    }
    return g;
}

lbib_status check_ligands(const lbib_ligand_desc& d, std::string& msg)
{
    if (d.rho_l_den <= 0 || d.rho_l_num < 0 || d.rho_l_num > d.rho_l_den)
        return msg = "ligand density must be a fraction in [0, 1]", LBIB_E_INVALID;
    const double v[] = {d.sigma_hat, d.sigma_star_ratio, d.y_cr_hat, d.y_eq_ratio,
                        d.k_f,       d.k_r0,             d.kbt_hat,  d.hamaker_hat};
    for (double x : v)
        if (!is_finite(x)) return msg = "non-finite parameter", LBIB_E_INVALID;
    if (d.sigma_hat < 0 || d.y_cr_hat < 0 || d.y_eq_ratio < 0 || d.k_f < 0 || d.k_r0 < 0 || d.hamaker_hat < 0)
        return msg = "negative rate, length or constant", LBIB_E_INVALID;
    if (!(d.kbt_hat > 0)) return msg = "kbt_hat must be > 0", LBIB_E_INVALID;
    return LBIB_OK;
}

void set_ligands(Particle& p, const lbib_ligand_desc& d)
{
    p.ligand = ligand_layout(p.nl, d.rho_l_num, d.rho_l_den);
    p.lig = d;
    p.has_ligands = true;
}

lbib_status prepare_particle(const lbib_lattice_desc& lat, const lbib_particle_desc& d, Particle& p, std::string& msg)
{
    if (d.shape != 0 && d.shape != 1) return msg = "shape must be 0 or 1", LBIB_E_INVALID;
    const double a = d.a_major, b = d.shape == 0 ? d.a_major : d.b_minor;
    if (!is_finite(a) || !is_finite(b) || !(a > 0) || !(b > 0)) return msg = "semi-axes must be positive", LBIB_E_INVALID;
    if (!is_finite(d.xc) || !is_finite(d.yc) || !is_finite(d.theta0)) return msg = "non-finite position", LBIB_E_INVALID;
    if (!is_finite(d.rho_p) || !(d.rho_p > 0)) return msg = "rho_p must be > 0", LBIB_E_INVALID;
    if (d.n_markers < 8 || d.n_markers > kMaxMarkers) return msg = "n_markers must be in [8, 1024]", LBIB_E_INVALID;
    const double amax = std::max(a, b);
    if (2.0 * amax + 6.0 > lat.nx) return msg = "particle too wide for the channel (2a + 6 > nx)", LBIB_E_INVALID;
    const double hs = support_h(a, b, d.theta0);
    if (!(d.yc - hs + 0.5 > 0.0) || !(d.yc + hs < lat.ny - 0.5))
        return msg = "particle must lie inside the channel with a positive gap", LBIB_E_INVALID;
    p.desc = d;
    p.nl = d.n_markers;
    p.a = a;
    p.b = b;
    if (!build_surface(d.shape, a, b, p.nl, p.surf)) return msg = "surface construction failed", LBIB_E_INVALID;
    if (p.surf.perimeter / p.nl < 0.25) return msg = "marker spacing below 0.25 lattice units", LBIB_E_INVALID;
    p.mass = d.rho_p * M_PI * a * b;
    p.inertia = p.mass * (a * a + b * b) / 4.0;
    // every marker lies within amax of the centroid and every probe within amax + 1.2; an
    // MLS support reaches 1.5 further, so any orientation's box has at most
    // ceil(2 amax + 2.4) + 4 nodes per side (one more kept as margin)
    const int side = (int)std::ceil(2.0 * amax + 2.4) + 5;
    if ((double)side * side > 1.0e6) return msg = "particle too large (box of more than 10^6 nodes)", LBIB_E_INVALID;
    p.box_cap = side * side;
    p.zone_side = side + 2 * kZoneMargin;  // the widened box's side at most
    if (!particle_lds_bytes(p.box_cap) && particle_lds_aux_bytes(p.box_cap) > 158 * 1024)
        return msg = "particle too large for the node mask in LDS", LBIB_E_INVALID;
    return LBIB_OK;
}

// The overlapped sweep's workgroups for the tiles of the particle's widened box: one per tile
// it can reach (Tile<PULL>), a multiple of 8, at most 64 (each then takes several): those that
// wait for the particle's force never hold so many CUs that its workgroup finds none.
int zone_workgroups(const Particle& p, bool pull)
{
    (void)pull;  // both layouts sweep 256 x 1 tiles
    const int tw = 256, th = 1, zs = p.zone_side;
    return std::min(64, (((zs + tw - 1) / tw + 1) * ((zs + th - 1) / th + 1) + 7) / 8 * 8);
}

size_t particle_block_bytes(const Particle& p)
{
    const size_t nl = (size_t)p.nl, cap = (size_t)p.box_cap;
    const size_t scratch = particle_scratch_bytes(p.box_cap);
    return 2 * align_up(2 * nl * 8) + align_up(nl * 8) + 2 * align_up(nl) + align_up(2 * cap * 8) +
           align_up((cap + 31) / 32 * 8) + (scratch ? align_up(scratch) : 0) + align_up(sizeof(TileDesc)) +
           align_up(2 * sizeof(TileDesc)) + align_up(16 * 8) + align_up(sizeof(DevParticle));
}

void carve_particle(Particle& p, char* block)
{
    const size_t nl = (size_t)p.nl, cap = (size_t)p.box_cap;
    char* c = block;
    auto take = [&](size_t bytes) {
        char* r = c;
        c += align_up(bytes);
        return r;
    };
    p.d_xi = (double*)take(2 * nl * 8);
    p.d_nuv = (double*)take(2 * nl * 8);
    p.d_S = (double*)take(nl * 8);
    p.d_lig = (uint8_t*)take(nl);
    p.d_bond = (uint8_t*)take(nl);
    p.d_tile = (int64_t*)take(2 * cap * 8);
    p.d_ring = (uint2*)take((cap + 31) / 32 * 8);
    const size_t scratch = particle_scratch_bytes(p.box_cap);
    p.d_box = scratch ? (double*)take(scratch) : nullptr;
    p.d_desc = (TileDesc*)take(sizeof(TileDesc));
    p.d_zone = (TileDesc*)take(2 * sizeof(TileDesc));
    p.d_count = (unsigned long long*)take(16 * 8);
    p.d_st = (DevParticle*)take(sizeof(DevParticle));
    p.block = block;
    p.own_block = false;
}

int64_t footprint_bytes(const lbib_lattice_desc& lat, const Particle* p)
{
    const LatticeGeom g = lattice_geom(lat);
    int64_t bytes = 2 * (int64_t)align_up(g.buf_bytes);
    if (p) bytes += (int64_t)particle_block_bytes(*p);
    return bytes;
}

hipError_t alloc_particle(Particle& p)
{
    char* block = nullptr;
    hipError_t e = hipMalloc((void**)&block, particle_block_bytes(p));
    if (e != hipSuccess) return e;
    carve_particle(p, block);
    p.own_block = true;
    return hipSuccess;
}

void free_particle(Particle& p)
{
    if (p.own_block && p.block) (void)hipFree(p.block);
    p.block = nullptr;
    p.own_block = false;
    p.d_xi = p.d_nuv = p.d_S = nullptr;
    p.d_lig = p.d_bond = nullptr;
    p.d_tile = nullptr;
    p.d_ring = nullptr;
    p.d_box = nullptr;
    p.d_desc = p.d_zone = nullptr;
    p.d_count = nullptr;
    p.d_st = nullptr;
    dfree(p.d_trace);
    p.trace_cap = 0;
}

hipError_t upload_particle(Particle& p, hipStream_t s)
{
    const int nl = p.nl;
    p.zeros.assign(nl, 0);
    DevParticle& st = p.st0;
    st = DevParticle{};
    st.xc = st.xc1 = p.desc.xc;
    st.yc = st.yc1 = p.desc.yc;
    st.th = st.th1 = p.desc.theta0;
    st.step = 0;
    st.last.step = -1;
    st.last.xc = st.xc;
    st.last.yc = st.yc;
    st.last.theta = st.th;
    st.last.gap = st.yc + 0.5 - support_h(p.a, p.b, st.th);
    p.td0[0] = p.td0[1] = TileDesc{};
    hipError_t e;
    if ((e = hipMemcpyAsync(p.d_zone, p.td0, 2 * sizeof(TileDesc), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p.d_xi, p.surf.xi.data(), 2 * nl * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p.d_nuv, p.surf.nu.data(), 2 * nl * sizeof(double), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(p.d_S, p.surf.S.data(), nl * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p.d_lig, p.ligand.data(), nl, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p.d_bond, p.zeros.data(), nl, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p.d_st, &p.st0, sizeof(DevParticle), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p.d_desc, p.td0, sizeof(TileDesc), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemsetAsync(p.d_count, 0, 16 * 8, s)) != hipSuccess)
        return e;
    return hipSuccess;
}

template <typename T>
void fill_particle_args(ParticleArgs<T>& a, const LatticeGeom& g, uint64_t seed, const Particle& p, int32_t* flags)
{
    a = ParticleArgs<T>{};
    a.target_steps = INT64_MAX;
    a.nx = g.nx;
    a.ny = g.ny;
    a.pitch = g.pitch;
    a.pull = g.pull ? 1 : 0;
    a.plane = g.plane;
    a.inv_scale = 1.0 / g.scale;
    a.uw6 = g.uw / 6.0;
    a.gx = g.gx;
    a.gy = g.gy;
    a.nu = g.nu;
    a.xi = p.d_xi;
    a.nuv = p.d_nuv;
    a.S = p.d_S;
    a.ligand = p.d_lig;
    a.bond = p.d_bond;
    a.nl = p.nl;
    a.a = p.a;
    a.b = p.b;
    a.mass = p.mass;
    a.inertia = p.inertia;
    // Table 1 dimensionless groups to lattice units (rho_ref = 1, length H = ny)
    const double H = (double)g.ny, nu2 = g.nu * g.nu;
    const lbib_ligand_desc& L = p.lig;
    a.sigma = L.sigma_hat * nu2 / H;
    a.sigma_star = L.sigma_star_ratio * a.sigma;
    a.y_cr = L.y_cr_hat * H;
    a.y_eq = L.y_eq_ratio * a.y_cr;
    a.k_f = L.k_f;
    a.k_r0 = L.k_r0;
    a.kBT = L.kbt_hat * nu2 * H;
    a.hamaker = L.hamaker_hat * nu2 * H;
    a.seed = seed;
    a.pid = 0;
    a.tile = p.d_tile;
    a.ring = p.d_ring;
    a.box_global = p.d_box;
    a.box_cap = p.box_cap;
    a.desc = p.d_desc;
    a.zone = p.d_zone;
    a.st = p.d_st;
    a.trace = p.d_trace;
    a.trace_cap = p.trace_cap;
    a.trace_start = p.trace_start;
    a.flags = flags;
}

template void fill_particle_args<float>(ParticleArgs<float>&, const LatticeGeom&, uint64_t, const Particle&, int32_t*);
template void fill_particle_args<double>(ParticleArgs<double>&, const LatticeGeom&, uint64_t, const Particle&,
                                         int32_t*);
template void fill_particle_args<half_t>(ParticleArgs<half_t>&, const LatticeGeom&, uint64_t, const Particle&,
                                         int32_t*);
template void fill_particle_args<bf16_t>(ParticleArgs<bf16_t>&, const LatticeGeom&, uint64_t, const Particle&,
                                         int32_t*);
template void fill_particle_args<half_neq_t>(ParticleArgs<half_neq_t>&, const LatticeGeom&, uint64_t, const Particle&,
                                             int32_t*);
template void fill_particle_args<bf16_neq_t>(ParticleArgs<bf16_neq_t>&, const LatticeGeom&, uint64_t, const Particle&,
                                             int32_t*);

// A lattice sweep reads one population buffer and writes the other.  Where the two together
// are at least twice the device's 256 MB last-level cache, odd steps take the tiles in reverse
// order, so that the first tiles a sweep reads are the last the previous sweep wrote
// (8192 x 4096, overlapped sweep: FP32 418 -> 397 us, FP16 225 -> 215, BF16 223 -> 215;
// 4096 x 1024 FP64, 604 MB: 94 -> 92).  Nearer the cache's size one order is as fast or faster
// (4096 x 1024 FP32, 302 MB: 44.9 against 46.6 us alternating), and the f - f_eq storages,
// whose buffers also hold the moments, measured slower alternating (8192 x 4096: 480 against
// 435 us), as did nothing for a pool of many small lattices (4 GB: 777 us either way), so
// both keep one order.  The order changes no result.
bool reverse_sweep(const LatticeGeom& g, int64_t step)
{
    constexpr size_t kLastLevelCache = (size_t)256 << 20;
    return (step & 1) != 0 && !g.neq && 2 * g.buf_bytes >= 2 * kLastLevelCache;
}

SweepArgs make_sweep_args(const LatticeGeom& g)
{
    SweepArgs a{};
    a.nx = g.nx;
    a.ny = g.ny;
    a.pitch = g.pitch;
    a.plane = g.plane;
    a.omega = 1.0 / g.tau;
    a.guo = 1.0 - 1.0 / (2.0 * g.tau);
    a.gx = g.gx;
    a.gy = g.gy;
    a.scale = g.scale;
    a.inv_scale = 1.0 / g.scale;
    a.uw6 = g.uw / 6.0;
    a.omega_f = (float)a.omega;
    a.keep_f = (float)(1.0 - a.omega);
    a.b3_f = (float)(3.0 * a.guo);
    a.b9_f = (float)(9.0 * a.guo);
    a.inv_scale_f = (float)a.inv_scale;
    return a;
}

hipError_t init_populations(void* f, const LatticeGeom& g, hipStream_t s)
{
    const size_t bytes = g.buf_bytes;
    hipError_t e = hipMemsetAsync(f, 0, bytes, s);
    if (e != hipSuccess) return e;
    switch (g.precision) {
        case LBIB_FP64: return launch_init<double>((double*)f, g.nx, g.ny, g.pitch, g.plane, g.umax, g.scale, g.pull, g.drive, s);
        case LBIB_FP32: return launch_init<float>((float*)f, g.nx, g.ny, g.pitch, g.plane, g.umax, g.scale, g.pull, g.drive, s);
        case LBIB_FP16: return launch_init<half_t>((half_t*)f, g.nx, g.ny, g.pitch, g.plane, g.umax, g.scale, g.pull, g.drive, s);
        case LBIB_BF16: return launch_init<bf16_t>((bf16_t*)f, g.nx, g.ny, g.pitch, g.plane, g.umax, g.scale, g.pull, g.drive, s);
        case LBIB_FP16_NEQ:
            return launch_init<half_neq_t>((half_neq_t*)f, g.nx, g.ny, g.pitch, g.plane, g.umax, g.scale, g.pull, g.drive, s);
        default:
            return launch_init<bf16_neq_t>((bf16_neq_t*)f, g.nx, g.ny, g.pitch, g.plane, g.umax, g.scale, g.pull, g.drive, s);
    }
}

// What a top-row population that arrives through the moving wall carries beyond the stored
// value (wall_reflect on the device): -u_w/6 for direction 7, +u_w/6 for 8.
static double wall_term(const LatticeGeom& g, int q)
{
    return q == 7 ? -g.uw / 6.0 : q == 8 ? g.uw / 6.0 : 0.0;
}

// Shifted equilibrium f_eq,q - w_q = w_q r_q of moments (drho, u), in the device's order of
// operations (feq_r): r_q = drho + rho (e.u (3 + 9/2 e.u) + P) with P = -3/2 u^2, e.u formed
// so that opposite directions give exact negatives.
static double feq_shift_host(int q, double drho, double ux, double uy)
{
    double eu = 0.0;
    switch (q) {
        case 1: eu = ux; break;
        case 2: eu = uy; break;
        case 3: eu = -ux; break;
        case 4: eu = -uy; break;
        case 5: eu = ux + uy; break;
        case 6: eu = uy - ux; break;
        case 7: eu = -(ux + uy); break;
        case 8: eu = ux - uy; break;
        default: break;
    }
    const double rho = 1.0 + drho, P = -1.5 * std::fma(ux, ux, uy * uy);
    const double r = q == 0 ? std::fma(rho, P, drho) : std::fma(rho, std::fma(eu, std::fma(4.5, eu, 3.0), P), drho);
    return kWq[q] * r;
}

// Non-equilibrium storages: the shifted equilibrium the reader of population q at (i, j)
// adds, from the stored moments m (moment k of node (i, j) at k plane + j mpitch + i) of the
// node that emitted it.
static double neq_term(const LatticeGeom& g, const float* m, int q, int i, int j)
{
    int si = i, sj = j, dir = q;
    const int jj = j - kEyq[q];
    if (jj < 0 || jj >= g.ny) {
        dir = kOppq[q];
    } else {
        si = i - kExq[q];
        si = si < 0 ? si + g.nx : (si >= g.nx ? si - g.nx : si);
        sj = jj;
    }
    const int64_t c = (int64_t)sj * g.mpitch + si;
    return feq_shift_host(dir, (double)m[c], (double)m[g.plane + c], (double)m[2 * g.plane + c]);
}

hipError_t download_populations(const void* fdev, const LatticeGeom& g, std::vector<double>& f)
{
    const int nx = g.nx, ny = g.ny;
    f.assign((size_t)9 * nx * ny, 0.0);
    std::vector<unsigned char> raw(g.buf_bytes);
    hipError_t e = hipMemcpy(raw.data(), fdev, raw.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    const float* mom = (const float*)(raw.data() + (size_t)9 * g.row * ny * g.elem);
    const double inv = 1.0 / g.scale;
    for (int q = 0; q < 9; ++q)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t k = host_pop_index(g, q, i, j);
                double v = 0.0;
                switch (g.precision) {
                    case LBIB_FP64: v = ((const double*)raw.data())[k]; break;
                    case LBIB_FP32: v = (double)((const float*)raw.data())[k]; break;
                    case LBIB_FP16:
                    case LBIB_FP16_NEQ: v = (double)f16_to_f32(((const uint16_t*)raw.data())[k]) * inv; break;
                    default: v = (double)bf16_to_f32(((const uint16_t*)raw.data())[k]); break;
                }
                if (g.neq) v += neq_term(g, mom, q, i, j);
                if (j == ny - 1) v += wall_term(g, q);
                f[((size_t)q * ny + j) * nx + i] = kWq[q] + v;
            }
    return hipSuccess;
}

hipError_t upload_populations(void* fdev, const LatticeGeom& g, const double* f)
{
    const int nx = g.nx, ny = g.ny;
    const size_t N = (size_t)nx * ny;
    std::vector<unsigned char> raw(g.buf_bytes, 0);
    float* mom = (float*)(raw.data() + (size_t)9 * g.row * ny * g.elem);
    if (g.neq) {
        // each node's moments (rho - 1, u) from the written populations: the equilibrium the
        // values it emits are stored against
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double r = 0.0, jx = 0.0, jy = 0.0;
                for (int q = 0; q < 9; ++q) {
                    const double v = f[(size_t)q * N + (size_t)j * nx + i];
                    r += v;
                    jx += v * kExq[q];
                    jy += v * kEyq[q];
                }
                const int64_t c = (int64_t)j * g.mpitch + i;
                mom[c] = (float)(r - 1.0);
                mom[g.plane + c] = (float)(jx / r);
                mom[2 * g.plane + c] = (float)(jy / r);
            }
    }
    for (int q = 0; q < 9; ++q)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t k = host_pop_index(g, q, i, j);
                double v = f[((size_t)q * ny + j) * nx + i] - kWq[q] - (j == ny - 1 ? wall_term(g, q) : 0.0);
                if (g.neq) v -= neq_term(g, mom, q, i, j);
                switch (g.precision) {
                    case LBIB_FP64: ((double*)raw.data())[k] = v; break;
                    case LBIB_FP32: ((float*)raw.data())[k] = (float)v; break;
                    case LBIB_FP16:
                    case LBIB_FP16_NEQ: ((uint16_t*)raw.data())[k] = f32_to_f16((float)v * (float)g.scale); break;
                    default: ((uint16_t*)raw.data())[k] = f32_to_bf16((float)v); break;
                }
            }
    return hipMemcpy(fdev, raw.data(), raw.size(), hipMemcpyHostToDevice);
}

void field_from_populations(const std::vector<double>& f, const LatticeGeom& g, int which, double* out)
{
    const size_t N = (size_t)g.nx * g.ny;
    if (which == 3) {
        std::memcpy(out, f.data(), f.size() * sizeof(double));
        return;
    }
    for (size_t c = 0; c < N; ++c) {
        double r = 0, jx = 0, jy = 0;
        for (int q = 0; q < 9; ++q) {
            const double v = f[q * N + c];
            r += v;
            jx += v * kExq[q];
            jy += v * kEyq[q];
        }
        out[c] = which == 0 ? r : which == 1 ? (jx + 0.5 * g.gx) / r : (jy + 0.5 * g.gy) / r;
    }
}

}  // namespace lbib
