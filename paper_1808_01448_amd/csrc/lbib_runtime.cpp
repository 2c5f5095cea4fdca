// lbib_runtime.cpp -- host side of the LB-IB adhesion library: argument validation, unit
// conversion (Table 1 groups to lattice units), device allocation, the per-step launch
// sequence, read-outs, checkpoints and kernel timing.  Implements include/lbib.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "lbib.h"
#include "lbib_geometry.hpp"
#include "lbib_internal.hpp"

using namespace lbib;

namespace {

constexpr double kWq[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                           1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
constexpr int kExq[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEyq[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

constexpr int kMaxMarkers = 1024;
constexpr int kTimingPool = 8192;  // event pairs per kernel kind

struct Particle {
    lbib_particle_desc desc{};
    lbib_ligand_desc lig{};
    bool has_ligands = false;
    int nl = 0;
    double a = 0, b = 0, mass = 0, inertia = 0;
    Surface surf;
    std::vector<uint8_t> ligand;
    // device
    double *d_xi = nullptr, *d_nuv = nullptr, *d_S = nullptr;
    uint8_t *d_lig = nullptr, *d_bond = nullptr;
    int64_t* d_tile = nullptr;
    double* d_box = nullptr;  // box node fields when they do not fit in LDS
    int box_cap = 0;
    TileDesc* d_desc = nullptr;
    TileDesc* d_zone = nullptr;  // two slots, by step parity
    DevParticle* d_st = nullptr;
    lbib_particle_state* d_trace = nullptr;
    int64_t trace_cap = 0, trace_start = 0;
};

constexpr int kKinds = 3;  // 0 lattice sweep (all or outside the box), 1 particle phase, 2 box sweep

struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev[kKinds];
    size_t used[kKinds] = {0, 0, 0};
    int64_t launches[kKinds] = {0, 0, 0};
};

}  // namespace

struct lbib_sim {
    lbib_lattice_desc desc{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t stream2 = nullptr;  // particle chain of the overlapped schedule
    hipEvent_t evA = nullptr, evB = nullptr;
    int overlap = 2;  // 0 serial, 1 overlapped, 2 chosen by lattice size
    bool zone_valid = false;  // the zone slot of the next step holds its box
    int state = 0;  // 0 created, 1 running, 2 failed
    std::string err;
    int pitch = 0;
    int64_t plane = 0;
    size_t elem = 0;
    void* fA = nullptr;
    void* fB = nullptr;
    double nu = 0, umax = 0, gx = 0, gy = 0;
    std::vector<Particle> parts;
    int32_t* d_flags = nullptr;
    int64_t steps = 0;
    Timing timing;
};

namespace {

thread_local std::string g_null_err;

lbib_status fail(lbib_sim* h, lbib_status s, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_null_err = msg;
    return s;
}

lbib_status hip_fail(lbib_sim* h, hipError_t e, const char* what)
{
    return fail(h, LBIB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                             \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call);      \
    } while (0)

bool is_finite(double v) { return std::isfinite(v); }

double support_h(double a, double b, double th)
{
    const double s = std::sin(th), c = std::cos(th);
    return std::sqrt(b * b * s * s + a * a * c * c);
}

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void free_particle(Particle& p)
{
    dfree(p.d_xi);
    dfree(p.d_nuv);
    dfree(p.d_S);
    dfree(p.d_lig);
    dfree(p.d_bond);
    dfree(p.d_tile);
    dfree(p.d_box);
    dfree(p.d_desc);
    dfree(p.d_zone);
    dfree(p.d_st);
    dfree(p.d_trace);
}

void free_all(lbib_sim* h)
{
    for (auto& p : h->parts) free_particle(p);
    if (h->fA) (void)hipFree(h->fA);
    if (h->fB) (void)hipFree(h->fB);
    h->fA = h->fB = nullptr;
    dfree(h->d_flags);
    for (int k = 0; k < kKinds; ++k) {
        for (auto e : h->timing.ev[k]) (void)hipEventDestroy(e);
        h->timing.ev[k].clear();
    }
    if (h->evA) (void)hipEventDestroy(h->evA);
    if (h->evB) (void)hipEventDestroy(h->evB);
    h->evA = h->evB = nullptr;
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
    h->stream2 = nullptr;
}

template <typename T>
hipError_t dalloc(T** p, size_t count)
{
    return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

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

template <typename T>
ParticleArgs<T> particle_args(lbib_sim* h, Particle& p)
{
    ParticleArgs<T> a{};
    a.f = (const T*)h->fA;
    a.nx = h->desc.nx;
    a.ny = h->desc.ny;
    a.pitch = h->pitch;
    a.plane = h->plane;
    a.gx = h->gx;
    a.gy = h->gy;
    a.nu = h->nu;
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
    const double H = (double)h->desc.ny, nu2 = h->nu * h->nu;
    const lbib_ligand_desc& L = p.lig;
    a.sigma = L.sigma_hat * nu2 / H;
    a.sigma_star = L.sigma_star_ratio * a.sigma;
    a.y_cr = L.y_cr_hat * H;
    a.y_eq = L.y_eq_ratio * a.y_cr;
    a.k_f = L.k_f;
    a.k_r0 = L.k_r0;
    a.kBT = L.kbt_hat * nu2 * H;
    a.hamaker = L.hamaker_hat * nu2 * H;
    a.seed = h->desc.seed;
    a.pid = 0;
    a.tile = p.d_tile;
    a.box_global = p.d_box;
    a.box_cap = p.box_cap;
    a.desc = p.d_desc;
    a.zone = p.d_zone;
    a.st = p.d_st;
    a.trace = p.d_trace;
    a.trace_cap = p.trace_cap;
    a.trace_start = p.trace_start;
    a.flags = h->d_flags;
    return a;
}

SweepArgs sweep_args(lbib_sim* h)
{
    SweepArgs a{};
    a.nx = h->desc.nx;
    a.ny = h->desc.ny;
    a.pitch = h->pitch;
    a.plane = h->plane;
    a.omega = 1.0 / h->desc.tau;
    a.guo = 1.0 - 1.0 / (2.0 * h->desc.tau);
    a.gx = h->gx;
    a.gy = h->gy;
    return a;
}

// Event pair that brackets the next launch of kernel `kind` (null when timing is off or the
// pool is used up).
struct EvPair {
    hipEvent_t t0 = nullptr, t1 = nullptr;
};

EvPair timing_events(lbib_sim* h, int kind)
{
    Timing& t = h->timing;
    EvPair p;
    if (!t.on || t.used[kind] + 2 > t.ev[kind].size()) return p;
    p.t0 = t.ev[kind][t.used[kind]];
    p.t1 = t.ev[kind][t.used[kind] + 1];
    t.used[kind] += 2;
    t.launches[kind] += 1;
    return p;
}

// One time step is the particle phase then the lattice sweep.  Serial schedule: both on the
// caller's stream.  Overlapped schedule (when the previous step has predicted this step's
// box): the particle phase runs on the second stream while the caller's stream sweeps the
// nodes outside the box (they carry no spread force); the box is swept after the particle
// phase.  Both schedules compute every node with the same arithmetic.
template <typename T>
lbib_status enqueue_steps(lbib_sim* h, int64_t n)
{
    const SweepArgs sa = sweep_args(h);
    bool joined = true;
    for (int64_t s = 0; s < n; ++s) {
        const T* fin = (const T*)h->fA;
        T* fout = (T*)h->fB;
        if (h->parts.empty()) {
            const EvPair e0 = timing_events(h, 0);
            HIPCHK(h, launch_sweep<T>(fin, fout, sa, SWEEP_ALL, nullptr, nullptr, 0, h->stream, e0.t0, e0.t1));
        } else {
            Particle& p = h->parts[0];
            ParticleArgs<T> pa = particle_args<T>(h, p);
            const int par = (int)(h->steps & 1);
            pa.parity_in = par;
            pa.parity_out = par ^ 1;
            // the overlapped schedule pays two cross-stream waits per step (~10 us); it wins
            // once a sweep moves more than ~64 MiB (the particle phase then hides behind it)
            const bool overlap =
                h->overlap == 1 || (h->overlap == 2 && (double)h->desc.nx * h->desc.ny * 18.0 * h->elem >= 64.0 * 1048576.0);
            if (!overlap || !h->zone_valid) {
                pa.check_zone = 0;
                const EvPair e1 = timing_events(h, 1);
                HIPCHK(h, launch_particle<T>(pa, h->stream, e1.t0, e1.t1));
                const EvPair e0 = timing_events(h, 0);
                HIPCHK(h, launch_sweep<T>(fin, fout, sa, SWEEP_ALL, p.d_desc, p.d_tile, p.box_cap, h->stream, e0.t0,
                                          e0.t1));
                HIPCHK(h, hipEventRecord(h->evA, h->stream));
                h->zone_valid = true;
            } else {
                pa.check_zone = 1;
                HIPCHK(h, hipStreamWaitEvent(h->stream2, h->evA, 0));
                const EvPair e1 = timing_events(h, 1);
                HIPCHK(h, launch_particle<T>(pa, h->stream2, e1.t0, e1.t1));
                HIPCHK(h, hipStreamWaitEvent(h->stream, h->evB, 0));
                const EvPair e0 = timing_events(h, 0);
                HIPCHK(h, launch_sweep<T>(fin, fout, sa, SWEEP_OUTSIDE, p.d_zone + par, nullptr, 0, h->stream, e0.t0,
                                          e0.t1));
                HIPCHK(h, hipEventRecord(h->evA, h->stream));
                const EvPair e2 = timing_events(h, 2);
                HIPCHK(h, launch_sweep<T>(fin, fout, sa, SWEEP_BOX, p.d_desc, p.d_tile, p.box_cap, h->stream2, e2.t0,
                                          e2.t1));
                HIPCHK(h, hipEventRecord(h->evB, h->stream2));
                joined = false;
            }
        }
        std::swap(h->fA, h->fB);
        h->steps += 1;
    }
    if (!joined) {
        // everything enqueued is ordered before later work on the caller's stream
        HIPCHK(h, hipStreamWaitEvent(h->stream, h->evB, 0));
        HIPCHK(h, hipEventRecord(h->evA, h->stream));
    }
    return LBIB_OK;
}

lbib_status check_flags(lbib_sim* h)
{
    int32_t fl = 0;
    HIPCHK(h, hipMemcpy(&fl, h->d_flags, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl) {
        h->state = 2;
        std::string m = "numerical failure:";
        if (fl & FLAG_NONFINITE) m += " non-finite force/torque/velocity;";
        if (fl & FLAG_CONTACT) m += " particle touches the receptor wall (gap <= 0);";
        if (fl & FLAG_MLS) m += " singular MLS moment matrix;";
        if (fl & FLAG_TILE) m += " spread footprint exceeds the tile;";
        return fail(h, LBIB_E_NUMERIC, m);
    }
    return LBIB_OK;
}

lbib_status sync_check(lbib_sim* h)
{
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return check_flags(h);
}

Particle* get_particle(lbib_sim* h, int32_t pid)
{
    if (pid < 0 || pid >= (int32_t)h->parts.size()) return nullptr;
    return &h->parts[pid];
}

// Populations on the device -> plain FP64 f (host, [9][ny][nx]).
lbib_status download_f(lbib_sim* h, std::vector<double>& f)
{
    const int nx = h->desc.nx, ny = h->desc.ny;
    const size_t n = (size_t)9 * h->plane;
    f.assign((size_t)9 * nx * ny, 0.0);
    if (h->elem == 8) {
        std::vector<double> raw(n);
        HIPCHK(h, hipMemcpy(raw.data(), h->fA, n * 8, hipMemcpyDeviceToHost));
        for (int q = 0; q < 9; ++q)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    f[((size_t)q * ny + j) * nx + i] = kWq[q] + raw[q * h->plane + (size_t)j * h->pitch + i];
    } else {
        std::vector<float> raw(n);
        HIPCHK(h, hipMemcpy(raw.data(), h->fA, n * 4, hipMemcpyDeviceToHost));
        for (int q = 0; q < 9; ++q)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    f[((size_t)q * ny + j) * nx + i] = kWq[q] + (double)raw[q * h->plane + (size_t)j * h->pitch + i];
    }
    return LBIB_OK;
}

struct BlobHeader {
    char magic[8];
    int32_t version, nx, ny, precision, n_particles, nl;
    int64_t steps, pop_bytes;
};

size_t blob_size(lbib_sim* h)
{
    size_t s = sizeof(BlobHeader) + (size_t)9 * h->plane * h->elem;
    for (auto& p : h->parts) s += sizeof(DevParticle) + (size_t)p.nl;
    return s;
}

}  // namespace

// ========================================================================================
// C-ABI
// ========================================================================================

extern "C" {

int lbib_abi_version(void) { return LBIB_ABI_VERSION; }

const char* lbib_last_error(lbib_handle h) { return h ? h->err.c_str() : g_null_err.c_str(); }

lbib_status lbib_create(const lbib_lattice_desc* d, void* hip_stream, lbib_handle* out)
{
    try {
        if (!d || !out) return fail(nullptr, LBIB_E_INVALID, "lbib_create: NULL argument");
        if (d->nx < 4 || d->ny < 4) return fail(nullptr, LBIB_E_INVALID, "lbib_create: nx and ny must be >= 4");
        if ((int64_t)d->nx * d->ny > (int64_t)1 << 31)
            return fail(nullptr, LBIB_E_INVALID, "lbib_create: more than 2^31 nodes");
        if (!is_finite(d->tau) || !(d->tau > 0.5)) return fail(nullptr, LBIB_E_INVALID, "lbib_create: tau must be > 1/2");
        if (!is_finite(d->re) || d->re < 0) return fail(nullptr, LBIB_E_INVALID, "lbib_create: Re must be >= 0");
        if (d->drive != 0)
            return fail(nullptr, LBIB_E_UNSUPPORTED, "lbib_create: only drive 0 (body-force Poiseuille) is built");
        if (d->precision != LBIB_FP64 && d->precision != LBIB_FP32)
            return fail(nullptr, LBIB_E_UNSUPPORTED, "lbib_create: precision must be LBIB_FP64 or LBIB_FP32");
        lbib_sim* h = new lbib_sim();
        h->desc = *d;
        if (hip_stream) {
            h->stream = (hipStream_t)hip_stream;
        } else {
            hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                delete h;
                return fail(nullptr, LBIB_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            }
            h->own_stream = true;
        }
        h->elem = d->precision == LBIB_FP64 ? 8 : 4;
        const int align = (int)(256 / h->elem);  // rows start on 256-byte boundaries
        h->pitch = (d->nx + align - 1) / align * align;
        h->plane = (int64_t)h->pitch * d->ny;
        const double H = (double)d->ny;
        h->nu = (d->tau - 0.5) / 3.0;
        h->umax = d->re * h->nu / H;
        h->gx = 8.0 * h->nu * h->umax / (H * H);
        h->gy = 0.0;
        *out = h;
        return LBIB_OK;
    } catch (const std::bad_alloc&) {
        return fail(nullptr, LBIB_E_NOMEM, "lbib_create: host allocation failed");
    } catch (...) {
        return fail(nullptr, LBIB_E_INVALID, "lbib_create: unexpected error");
    }
}

lbib_status lbib_particle_add(lbib_handle h, const lbib_particle_desc* d, int32_t* pid)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_particle_add: NULL handle");
    try {
        if (!d || !pid) return fail(h, LBIB_E_INVALID, "lbib_particle_add: NULL argument");
        if (h->state != 0) return fail(h, LBIB_E_STATE, "lbib_particle_add: must precede lbib_init");
        if (!h->parts.empty()) return fail(h, LBIB_E_UNSUPPORTED, "lbib_particle_add: one particle per simulation");
        if (d->shape != 0 && d->shape != 1) return fail(h, LBIB_E_INVALID, "lbib_particle_add: shape must be 0 or 1");
        const double a = d->a_major, b = d->shape == 0 ? d->a_major : d->b_minor;
        if (!is_finite(a) || !is_finite(b) || !(a > 0) || !(b > 0))
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: semi-axes must be positive");
        if (!is_finite(d->xc) || !is_finite(d->yc) || !is_finite(d->theta0))
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: non-finite position");
        if (!is_finite(d->rho_p) || !(d->rho_p > 0)) return fail(h, LBIB_E_INVALID, "lbib_particle_add: rho_p must be > 0");
        if (d->n_markers < 8 || d->n_markers > kMaxMarkers)
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: n_markers must be in [8, 1024]");
        const double amax = std::max(a, b);
        if (2.0 * amax + 6.0 > h->desc.nx)
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: particle too wide for the channel (2a + 6 > nx)");
        const double hs = support_h(a, b, d->theta0);
        if (!(d->yc - hs + 0.5 > 0.0) || !(d->yc + hs < h->desc.ny - 0.5))
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: particle must lie inside the channel with a positive gap");
        Particle p;
        p.desc = *d;
        p.nl = d->n_markers;
        p.a = a;
        p.b = b;
        if (!build_surface(d->shape, a, b, p.nl, p.surf))
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: surface construction failed");
        if (p.surf.perimeter / p.nl < 0.25)
            return fail(h, LBIB_E_INVALID, "lbib_particle_add: marker spacing below 0.25 lattice units");
        p.mass = d->rho_p * M_PI * a * b;
        p.inertia = p.mass * (a * a + b * b) / 4.0;
        // every marker lies within amax of the centroid and every probe within amax + 1.2;
        // an MLS support reaches 1.5 further, so any orientation's box has at most
        // ceil(2 amax + 2.4) + 4 nodes per side (one more kept as margin)
        const int side = (int)std::ceil(2.0 * amax + 2.4) + 5;
        p.box_cap = side * side;
        h->parts.push_back(std::move(p));
        *pid = (int32_t)h->parts.size() - 1;
        return LBIB_OK;
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_particle_add: host allocation failed");
    }
}

lbib_status lbib_ligands_set(lbib_handle h, int32_t pid, const lbib_ligand_desc* d)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_ligands_set: NULL handle");
    if (!d) return fail(h, LBIB_E_INVALID, "lbib_ligands_set: NULL descriptor");
    if (h->state != 0) return fail(h, LBIB_E_STATE, "lbib_ligands_set: must precede lbib_init");
    Particle* p = get_particle(h, pid);
    if (!p) return fail(h, LBIB_E_INVALID, "lbib_ligands_set: unknown particle id");
    if (d->rho_l_den <= 0 || d->rho_l_num < 0 || d->rho_l_num > d->rho_l_den)
        return fail(h, LBIB_E_INVALID, "lbib_ligands_set: ligand density must be a fraction in [0, 1]");
    const double v[] = {d->sigma_hat, d->sigma_star_ratio, d->y_cr_hat, d->y_eq_ratio,
                        d->k_f,       d->k_r0,             d->kbt_hat,  d->hamaker_hat};
    for (double x : v)
        if (!is_finite(x)) return fail(h, LBIB_E_INVALID, "lbib_ligands_set: non-finite parameter");
    if (d->sigma_hat < 0 || d->y_cr_hat < 0 || d->y_eq_ratio < 0 || d->k_f < 0 || d->k_r0 < 0 || d->hamaker_hat < 0)
        return fail(h, LBIB_E_INVALID, "lbib_ligands_set: negative rate, length or constant");
    if (!(d->kbt_hat > 0)) return fail(h, LBIB_E_INVALID, "lbib_ligands_set: kbt_hat must be > 0");
    try {
        p->ligand = ligand_layout(p->nl, d->rho_l_num, d->rho_l_den);
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_ligands_set: host allocation failed");
    }
    p->lig = *d;
    p->has_ligands = true;
    return LBIB_OK;
}

lbib_status lbib_receptors_set(lbib_handle h, const lbib_receptor_desc* d)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_receptors_set: NULL handle");
    if (!d) return fail(h, LBIB_E_INVALID, "lbib_receptors_set: NULL descriptor");
    if (h->state != 0) return fail(h, LBIB_E_STATE, "lbib_receptors_set: must precede lbib_init");
    if (d->wall != 0 || d->density != 1.0)
        return fail(h, LBIB_E_UNSUPPORTED, "lbib_receptors_set: only full coverage (density 1) of the bottom wall");
    return LBIB_OK;
}

lbib_status lbib_init(lbib_handle h)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_init: NULL handle");
    if (h->state != 0) return fail(h, LBIB_E_STATE, "lbib_init: already initialised");
    for (auto& p : h->parts)
        if (!p.has_ligands) return fail(h, LBIB_E_STATE, "lbib_init: lbib_ligands_set missing for a particle");
    const int nx = h->desc.nx, ny = h->desc.ny;
    const size_t bytes = (size_t)9 * h->plane * h->elem;
    hipError_t e;
    if ((e = hipMalloc(&h->fA, bytes)) != hipSuccess || (e = hipMalloc(&h->fB, bytes)) != hipSuccess ||
        (e = dalloc(&h->d_flags, 1)) != hipSuccess) {
        free_all(h);
        return fail(h, e == hipErrorOutOfMemory ? LBIB_E_NOMEM : LBIB_E_DEVICE,
                    std::string("lbib_init: device allocation: ") + hipGetErrorString(e));
    }
    for (auto& p : h->parts) {
        const int nl = p.nl;
        const size_t tile = (size_t)2 * p.box_cap;
        const size_t boxg = particle_lds_bytes(p.box_cap) ? 0 : (size_t)6 * p.box_cap;
        if ((e = dalloc(&p.d_xi, 2 * nl)) != hipSuccess || (e = dalloc(&p.d_nuv, 2 * nl)) != hipSuccess ||
            (e = dalloc(&p.d_S, nl)) != hipSuccess || (e = dalloc(&p.d_lig, nl)) != hipSuccess ||
            (e = dalloc(&p.d_bond, nl)) != hipSuccess || (e = dalloc(&p.d_tile, tile)) != hipSuccess ||
            (boxg && (e = dalloc(&p.d_box, boxg)) != hipSuccess) || (e = dalloc(&p.d_zone, 2)) != hipSuccess || (e = dalloc(&p.d_desc, 1)) != hipSuccess ||
            (e = dalloc(&p.d_st, 1)) != hipSuccess) {
            free_all(h);
            return fail(h, e == hipErrorOutOfMemory ? LBIB_E_NOMEM : LBIB_E_DEVICE,
                        std::string("lbib_init: device allocation: ") + hipGetErrorString(e));
        }
    }
    auto bail = [&](hipError_t err, const char* what) {
        free_all(h);
        return hip_fail(h, err, what);
    };
    if ((e = hipMemsetAsync(h->fA, 0, bytes, h->stream)) != hipSuccess) return bail(e, "hipMemset");
    if ((e = hipMemsetAsync(h->fB, 0, bytes, h->stream)) != hipSuccess) return bail(e, "hipMemset");
    if ((e = hipMemsetAsync(h->d_flags, 0, sizeof(int32_t), h->stream)) != hipSuccess) return bail(e, "hipMemset");
    if (h->elem == 8)
        e = launch_init<double>((double*)h->fA, nx, ny, h->pitch, h->plane, h->umax, h->stream);
    else
        e = launch_init<float>((float*)h->fA, nx, ny, h->pitch, h->plane, h->umax, h->stream);
    if (e != hipSuccess) return bail(e, "init kernel");
    for (auto& p : h->parts) {
        const int nl = p.nl;
        std::vector<uint8_t> zeros(nl, 0);
        DevParticle st{};
        st.xc = st.xc1 = p.desc.xc;
        st.yc = st.yc1 = p.desc.yc;
        st.th = st.th1 = p.desc.theta0;
        st.step = 0;
        st.last.step = -1;
        st.last.xc = st.xc;
        st.last.yc = st.yc;
        st.last.theta = st.th;
        st.last.gap = st.yc + 0.5 - support_h(p.a, p.b, st.th);
        TileDesc td[2] = {};
        if ((e = hipMemcpy(p.d_zone, td, sizeof(td), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_xi, p.surf.xi.data(), 2 * nl * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_nuv, p.surf.nu.data(), 2 * nl * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_S, p.surf.S.data(), nl * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_lig, p.ligand.data(), nl, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_bond, zeros.data(), nl, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_st, &st, sizeof(st), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p.d_desc, td, sizeof(TileDesc), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "lbib_init: upload");
    }
    if ((e = hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking)) != hipSuccess)
        return bail(e, "lbib_init: second stream");
    if ((e = hipEventCreateWithFlags(&h->evA, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->evB, hipEventDisableTiming)) != hipSuccess)
        return bail(e, "lbib_init: events");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return bail(e, "lbib_init: sync");
    h->state = 1;
    h->steps = 0;
    h->zone_valid = false;
    return LBIB_OK;
}

lbib_status lbib_step(lbib_handle h, int64_t n)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_step: NULL handle");
    if (n < 0) return fail(h, LBIB_E_INVALID, "lbib_step: negative step count");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_step: lbib_init first");
    if (h->state == 2) return fail(h, LBIB_E_STATE, "lbib_step: simulation failed; lbib_load a good state");
    if (h->elem == 8) return enqueue_steps<double>(h, n);
    return enqueue_steps<float>(h, n);
}

lbib_status lbib_sync(lbib_handle h)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_sync: NULL handle");
    if (h->state == 0) return LBIB_OK;
    return sync_check(h);
}

lbib_status lbib_step_count(lbib_handle h, int64_t* steps)
{
    if (!h || !steps) return fail(h, LBIB_E_INVALID, "lbib_step_count: NULL argument");
    *steps = h->steps;
    return LBIB_OK;
}

lbib_status lbib_read_particle(lbib_handle h, int32_t pid, lbib_particle_state* out)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_read_particle: NULL handle");
    if (!out) return fail(h, LBIB_E_INVALID, "lbib_read_particle: NULL output");
    Particle* p = get_particle(h, pid);
    if (!p) return fail(h, LBIB_E_INVALID, "lbib_read_particle: unknown particle id");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_read_particle: lbib_init first");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    DevParticle st;
    HIPCHK(h, hipMemcpy(&st, p->d_st, sizeof(st), hipMemcpyDeviceToHost));
    *out = st.last;
    return check_flags(h);
}

lbib_status lbib_read_bonds(lbib_handle h, int32_t pid, uint8_t* bonded, uint8_t* ligand, int32_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_read_bonds: NULL handle");
    Particle* p = get_particle(h, pid);
    if (!p) return fail(h, LBIB_E_INVALID, "lbib_read_bonds: unknown particle id");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_read_bonds: lbib_init first");
    if (capacity < p->nl) return fail(h, LBIB_E_INVALID, "lbib_read_bonds: capacity must be >= " + std::to_string(p->nl));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (bonded) HIPCHK(h, hipMemcpy(bonded, p->d_bond, p->nl, hipMemcpyDeviceToHost));
    if (ligand) std::memcpy(ligand, p->ligand.data(), p->nl);
    return check_flags(h);
}

lbib_status lbib_read_markers(lbib_handle h, int32_t pid, double* xy, double* nxy, int32_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_read_markers: NULL handle");
    Particle* p = get_particle(h, pid);
    if (!p) return fail(h, LBIB_E_INVALID, "lbib_read_markers: unknown particle id");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_read_markers: lbib_init first");
    if (capacity < p->nl)
        return fail(h, LBIB_E_INVALID, "lbib_read_markers: capacity must be >= " + std::to_string(p->nl));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    DevParticle st;
    HIPCHK(h, hipMemcpy(&st, p->d_st, sizeof(st), hipMemcpyDeviceToHost));
    const double c = std::cos(st.th), s = std::sin(st.th);
    for (int l = 0; l < p->nl; ++l) {
        const double bx = p->surf.xi[2 * l], by = p->surf.xi[2 * l + 1];
        const double mx = p->surf.nu[2 * l], my = p->surf.nu[2 * l + 1];
        if (xy) {
            xy[2 * l] = st.xc + c * bx - s * by;
            xy[2 * l + 1] = st.yc + s * bx + c * by;
        }
        if (nxy) {
            nxy[2 * l] = c * mx - s * my;
            nxy[2 * l + 1] = s * mx + c * my;
        }
    }
    return check_flags(h);
}

lbib_status lbib_read_field(lbib_handle h, int32_t which, double* out, int64_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_read_field: NULL handle");
    if (!out) return fail(h, LBIB_E_INVALID, "lbib_read_field: NULL output");
    if (which < 0 || which > 3) return fail(h, LBIB_E_INVALID, "lbib_read_field: which must be 0..3");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_read_field: lbib_init first");
    const int nx = h->desc.nx, ny = h->desc.ny;
    const int64_t need = (which == 3 ? 9 : 1) * (int64_t)nx * ny;
    if (capacity < need) return fail(h, LBIB_E_INVALID, "lbib_read_field: capacity must be >= " + std::to_string(need));
    try {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        std::vector<double> f;
        lbib_status s = download_f(h, f);
        if (s != LBIB_OK) return s;
        if (which == 3) {
            std::memcpy(out, f.data(), f.size() * sizeof(double));
        } else {
            const size_t N = (size_t)nx * ny;
            for (size_t c = 0; c < N; ++c) {
                double r = 0, jx = 0, jy = 0;
                for (int q = 0; q < 9; ++q) {
                    const double v = f[q * N + c];
                    r += v;
                    jx += v * kExq[q];
                    jy += v * kEyq[q];
                }
                out[c] = which == 0 ? r : which == 1 ? (jx + 0.5 * h->gx) / r : (jy + 0.5 * h->gy) / r;
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_read_field: host allocation failed");
    }
    return check_flags(h);
}

lbib_status lbib_write_populations(lbib_handle h, const double* f, int64_t count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_write_populations: NULL handle");
    if (!f) return fail(h, LBIB_E_INVALID, "lbib_write_populations: NULL input");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_write_populations: lbib_init first");
    const int nx = h->desc.nx, ny = h->desc.ny;
    if (count != (int64_t)9 * nx * ny)
        return fail(h, LBIB_E_INVALID, "lbib_write_populations: count must be 9 nx ny");
    try {
        const size_t n = (size_t)9 * h->plane;
        HIPCHK(h, hipStreamSynchronize(h->stream));
        if (h->elem == 8) {
            std::vector<double> raw(n, 0.0);
            for (int q = 0; q < 9; ++q)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i)
                        raw[q * h->plane + (size_t)j * h->pitch + i] = f[((size_t)q * ny + j) * nx + i] - kWq[q];
            HIPCHK(h, hipMemcpy(h->fA, raw.data(), n * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> raw(n, 0.0f);
            for (int q = 0; q < 9; ++q)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i)
                        raw[q * h->plane + (size_t)j * h->pitch + i] =
                            (float)(f[((size_t)q * ny + j) * nx + i] - kWq[q]);
            HIPCHK(h, hipMemcpy(h->fA, raw.data(), n * 4, hipMemcpyHostToDevice));
        }
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_write_populations: host allocation failed");
    }
    return LBIB_OK;
}

lbib_status lbib_write_particle(lbib_handle h, int32_t pid, const double* v)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_write_particle: NULL handle");
    Particle* p = get_particle(h, pid);
    if (!p || !v) return fail(h, LBIB_E_INVALID, "lbib_write_particle: unknown particle or NULL input");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_write_particle: lbib_init first");
    for (int k = 0; k < 12; ++k)
        if (!is_finite(v[k])) return fail(h, LBIB_E_INVALID, "lbib_write_particle: non-finite value");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    DevParticle st;
    HIPCHK(h, hipMemcpy(&st, p->d_st, sizeof(st), hipMemcpyDeviceToHost));
    st.xc = v[0];
    st.yc = v[1];
    st.th = v[2];
    st.ux = v[3];
    st.uy = v[4];
    st.om = v[5];
    st.xc1 = v[6];
    st.yc1 = v[7];
    st.th1 = v[8];
    st.ux1 = v[9];
    st.uy1 = v[10];
    st.om1 = v[11];
    HIPCHK(h, hipMemcpy(p->d_st, &st, sizeof(st), hipMemcpyHostToDevice));
    h->zone_valid = false;  // the predicted box no longer matches the particle
    return LBIB_OK;
}

lbib_status lbib_write_bonds(lbib_handle h, int32_t pid, const uint8_t* bonded, int32_t count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_write_bonds: NULL handle");
    Particle* p = get_particle(h, pid);
    if (!p || !bonded) return fail(h, LBIB_E_INVALID, "lbib_write_bonds: unknown particle or NULL input");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_write_bonds: lbib_init first");
    if (count != p->nl) return fail(h, LBIB_E_INVALID, "lbib_write_bonds: count must equal n_markers");
    for (int l = 0; l < p->nl; ++l)
        if (bonded[l] > 1 || (bonded[l] && !p->ligand[l]))
            return fail(h, LBIB_E_INVALID, "lbib_write_bonds: flags must be 0/1 and only on ligand elements");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(p->d_bond, bonded, p->nl, hipMemcpyHostToDevice));
    return LBIB_OK;
}

lbib_status lbib_trace_enable(lbib_handle h, int32_t pid, int64_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_trace_enable: NULL handle");
    Particle* p = get_particle(h, pid);
    if (!p) return fail(h, LBIB_E_INVALID, "lbib_trace_enable: unknown particle id");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_trace_enable: lbib_init first");
    if (capacity < 0 || capacity > ((int64_t)1 << 28))
        return fail(h, LBIB_E_INVALID, "lbib_trace_enable: capacity must be in [0, 2^28]");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    dfree(p->d_trace);
    p->trace_cap = 0;
    if (capacity > 0) {
        hipError_t e = dalloc(&p->d_trace, (size_t)capacity);
        if (e != hipSuccess) return hip_fail(h, e, "lbib_trace_enable: allocation");
        p->trace_cap = capacity;
    }
    p->trace_start = h->steps;
    return LBIB_OK;
}

lbib_status lbib_read_trace(lbib_handle h, int32_t pid, lbib_particle_state* out, int64_t capacity, int64_t* count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_read_trace: NULL handle");
    Particle* p = get_particle(h, pid);
    if (!p || !out || !count) return fail(h, LBIB_E_INVALID, "lbib_read_trace: unknown particle or NULL output");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_read_trace: lbib_init first");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int64_t have = std::min(p->trace_cap, std::max<int64_t>(0, h->steps - p->trace_start));
    const int64_t n = std::min(have, capacity);
    if (n > 0) HIPCHK(h, hipMemcpy(out, p->d_trace, (size_t)n * sizeof(lbib_particle_state), hipMemcpyDeviceToHost));
    *count = n;
    return check_flags(h);
}

lbib_status lbib_save(lbib_handle h, void* blob, int64_t* size)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_save: NULL handle");
    if (!size) return fail(h, LBIB_E_INVALID, "lbib_save: NULL size");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_save: lbib_init first");
    const size_t need = blob_size(h);
    if (!blob) {
        *size = (int64_t)need;
        return LBIB_OK;
    }
    if (*size < (int64_t)need) return fail(h, LBIB_E_INVALID, "lbib_save: blob must hold " + std::to_string(need) + " bytes");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    char* w = (char*)blob;
    BlobHeader hd{};
    std::memcpy(hd.magic, "LBIBCKP1", 8);
    hd.version = LBIB_ABI_VERSION;
    hd.nx = h->desc.nx;
    hd.ny = h->desc.ny;
    hd.precision = h->desc.precision;
    hd.n_particles = (int32_t)h->parts.size();
    hd.nl = h->parts.empty() ? 0 : h->parts[0].nl;
    hd.steps = h->steps;
    hd.pop_bytes = (int64_t)9 * h->plane * (int64_t)h->elem;
    std::memcpy(w, &hd, sizeof(hd));
    w += sizeof(hd);
    HIPCHK(h, hipMemcpy(w, h->fA, (size_t)hd.pop_bytes, hipMemcpyDeviceToHost));
    w += hd.pop_bytes;
    for (auto& p : h->parts) {
        HIPCHK(h, hipMemcpy(w, p.d_st, sizeof(DevParticle), hipMemcpyDeviceToHost));
        w += sizeof(DevParticle);
        HIPCHK(h, hipMemcpy(w, p.d_bond, p.nl, hipMemcpyDeviceToHost));
        w += p.nl;
    }
    *size = (int64_t)need;
    return check_flags(h);
}

lbib_status lbib_load(lbib_handle h, const void* blob, int64_t size)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_load: NULL handle");
    if (!blob) return fail(h, LBIB_E_INVALID, "lbib_load: NULL blob");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_load: lbib_init first");
    if (size != (int64_t)blob_size(h)) return fail(h, LBIB_E_INVALID, "lbib_load: blob size does not match this simulation");
    BlobHeader hd;
    std::memcpy(&hd, blob, sizeof(hd));
    if (std::memcmp(hd.magic, "LBIBCKP1", 8) != 0 || hd.version != LBIB_ABI_VERSION || hd.nx != h->desc.nx ||
        hd.ny != h->desc.ny || hd.precision != h->desc.precision || hd.n_particles != (int32_t)h->parts.size() ||
        (hd.n_particles && hd.nl != h->parts[0].nl) || hd.pop_bytes != (int64_t)9 * h->plane * (int64_t)h->elem)
        return fail(h, LBIB_E_INVALID, "lbib_load: checkpoint was made with different descriptors");
    const char* r = (const char*)blob + sizeof(hd);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(h->fA, r, (size_t)hd.pop_bytes, hipMemcpyHostToDevice));
    r += hd.pop_bytes;
    for (auto& p : h->parts) {
        HIPCHK(h, hipMemcpy(p.d_st, r, sizeof(DevParticle), hipMemcpyHostToDevice));
        r += sizeof(DevParticle);
        HIPCHK(h, hipMemcpy(p.d_bond, r, p.nl, hipMemcpyHostToDevice));
        r += p.nl;
        p.trace_start = hd.steps;  // a trace restarts at the restored step
    }
    const int32_t zero = 0;
    HIPCHK(h, hipMemcpy(h->d_flags, &zero, sizeof(zero), hipMemcpyHostToDevice));
    h->steps = hd.steps;
    h->state = 1;
    h->zone_valid = false;
    return LBIB_OK;
}

lbib_status lbib_kernel_timing(lbib_handle h, int32_t enable)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_timing: NULL handle");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    Timing& t = h->timing;
    if (enable) {
        for (int k = 0; k < kKinds; ++k) {
            while (t.ev[k].size() < (size_t)2 * kTimingPool) {
                hipEvent_t e;
                HIPCHK(h, hipEventCreate(&e));
                t.ev[k].push_back(e);
            }
            t.used[k] = 0;
            t.launches[k] = 0;
        }
    }
    t.on = enable != 0;
    return LBIB_OK;
}

lbib_status lbib_kernel_time(lbib_handle h, int32_t kernel, double* total_ms, int64_t* launches)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_time: NULL handle");
    if (kernel < 0 || kernel >= kKinds || !total_ms || !launches)
        return fail(h, LBIB_E_INVALID, "lbib_kernel_time: kernel must be 0, 1 or 2 and outputs non-NULL");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    Timing& t = h->timing;
    double acc = 0.0;
    for (size_t k = 0; k + 1 < t.used[kernel]; k += 2) {
        float ms = 0.0f;
        HIPCHK(h, hipEventElapsedTime(&ms, t.ev[kernel][k], t.ev[kernel][k + 1]));
        acc += ms;
    }
    *total_ms = acc;
    *launches = t.launches[kernel];
    return LBIB_OK;
}

lbib_status lbib_set_overlap(lbib_handle h, int32_t mode)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_set_overlap: NULL handle");
    if (mode < 0 || mode > 2) return fail(h, LBIB_E_INVALID, "lbib_set_overlap: mode must be 0, 1 or 2");
    h->overlap = mode;
    return LBIB_OK;
}

lbib_status lbib_bytes_per_update(lbib_handle h, int64_t* bytes)
{
    if (!h || !bytes) return fail(h, LBIB_E_INVALID, "lbib_bytes_per_update: NULL argument");
    *bytes = (int64_t)(18 * h->elem);
    return LBIB_OK;
}

void lbib_destroy(lbib_handle h)
{
    if (!h) return;
    // nothing is enqueued before lbib_init, so an uninitialised handle never touches the GPU
    if (h->state != 0 && h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->state != 0) free_all(h);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

// ---------------------------------------------------------------------------------------
// Kernel-level entry points
// ---------------------------------------------------------------------------------------

lbib_status lbib_kernel_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n, void* s)
{
    if (n < 0 || n > 0x7fffffff) return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_philox: n out of range");
    if (n > 0 && (!ctr || !key || !out)) return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_philox: NULL buffer");
    hipError_t e = launch_philox(ctr, key, out, n, (hipStream_t)s);
    return e == hipSuccess ? LBIB_OK : hip_fail(nullptr, e, "lbib_kernel_philox");
}

lbib_status lbib_kernel_mls(const double* pts, int64_t n, int32_t nx, int32_t ny, int32_t* node, double* phi,
                            double* psix, double* psiy, void* s)
{
    if (n < 0 || n > 0x7fffffff || nx < 4 || ny < 4)
        return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_mls: bad size");
    if (n > 0 && (!pts || !node || !phi || !psix || !psiy))
        return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_mls: NULL buffer");
    hipError_t e = launch_mls(pts, n, nx, ny, node, phi, psix, psiy, (hipStream_t)s);
    return e == hipSuccess ? LBIB_OK : hip_fail(nullptr, e, "lbib_kernel_mls");
}

lbib_status lbib_kernel_bonds(const uint8_t* ligand, const double* d, const uint8_t* b_in, uint8_t* b_out,
                              const int64_t* step, int32_t* n_bonds, int32_t* n_probing, int32_t nl, int32_t n_sets,
                              const double* params, uint64_t seed, uint32_t pid, void* s)
{
    if (nl < 1 || nl > 65536 || n_sets < 0 || n_sets > 0x7fffffff || !params)
        return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_bonds: bad size or NULL params");
    if (n_sets > 0 && (!ligand || !d || !b_in || !b_out || !step || !n_bonds || !n_probing))
        return fail(nullptr, LBIB_E_INVALID, "lbib_kernel_bonds: NULL buffer");
    hipError_t e = launch_bonds(ligand, d, b_in, b_out, step, n_bonds, n_probing, nl, n_sets, params, seed, pid,
                                (hipStream_t)s);
    return e == hipSuccess ? LBIB_OK : hip_fail(nullptr, e, "lbib_kernel_bonds");
}

lbib_status lbib_bandwidth_probe(int64_t bytes, int32_t iters, void* s, double* gbps)
{
    if (bytes < 16 || bytes % 16 != 0 || iters < 1 || !gbps)
        return fail(nullptr, LBIB_E_INVALID, "lbib_bandwidth_probe: bytes must be a positive multiple of 16");
    hipStream_t st = (hipStream_t)s;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    double best = 0.0;
    if ((e = hipMalloc(&a, (size_t)bytes)) != hipSuccess || (e = hipMalloc(&b, (size_t)bytes)) != hipSuccess) goto out;
    if ((e = hipMemsetAsync(a, 1, (size_t)bytes, st)) != hipSuccess) goto out;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) goto out;
    if ((e = launch_copy((const float4*)a, (float4*)b, bytes / 16, st)) != hipSuccess) goto out;
    for (int k = 0; k < iters; ++k) {
        float ms = 0.0f;
        if ((e = hipEventRecord(e0, st)) != hipSuccess) goto out;
        if ((e = launch_copy((const float4*)a, (float4*)b, bytes / 16, st)) != hipSuccess) goto out;
        if ((e = hipEventRecord(e1, st)) != hipSuccess) goto out;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) goto out;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) goto out;
        if (ms > 0) best = std::max(best, 2.0 * (double)bytes / (ms * 1e-3) / 1e9);
    }
out:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e != hipSuccess) return hip_fail(nullptr, e, "lbib_bandwidth_probe");
    *gbps = best;
    return LBIB_OK;
}

}  // extern "C"
