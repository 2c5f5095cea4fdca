// lbib_static.hip -- lbib_solve_static: one particle in one channel, advanced with the serial
// schedule (particle phase, then the sweep of every node, per step), without allocating device
// memory.  The caller passes the population buffers and the outputs; every other device buffer
// the library would allocate for the solve (the particle's surface, ligand and bond flags,
// spread-force tile and its index, box descriptors, hand-over words, node-field overflow,
// rigid-body state and the watchdog word) is carved from `scratch`, one static array per GPU.
// The kernels are those of lbib_step, so a solve gives the same results bit for bit as the
// handle-based calls with the serial schedule.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lbib.h"
#include "lbib_host.hpp"
#include "lbib_internal.hpp"

namespace lbib {

// Size of the static area on each GPU: a particle whose buffers (particle_block_bytes, set by
// its marker count and the side of its box) need more is refused.  8 MiB holds any particle
// of up to 1024 markers whose box side stays below about 350 nodes (semi-axes up to about 170).
constexpr size_t kStaticScratchBytes = size_t(8) << 20;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

// Per device: the device address of `scratch` (looked up once, with the device current) and a
// lock held for the whole of a solve, so calls from several host threads on one GPU take the
// array one after the other instead of overlapping on it.
struct StaticArea {
    std::mutex mu;
    void* ptr = nullptr;
};
StaticArea g_area[kMaxDevices];

hipError_t area_address(int dev, void** out)
{
    StaticArea& a = g_area[dev];
    if (!a.ptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        a.ptr = p;
    }
    *out = a.ptr;
    return hipSuccess;
}

lbib_status fail(lbib_status s, const std::string& msg)
{
    set_null_error("lbib_solve_static: " + msg);
    return s;
}

lbib_status hip_fail(hipError_t e, const char* what)
{
    return fail(LBIB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define SCHK(call)                                             \
    do {                                                       \
        const hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

// Enqueue the initial state and n serial steps on s (fA holds level 0 on return of the
// enqueue; the buffers swap every step, as in lbib_step).
template <typename T>
lbib_status enqueue_solve(const LatticeGeom& g, uint64_t seed, Particle& p, int64_t n, char* fA, char* fB,
                          lbib_particle_state* trace, int32_t* flags, hipStream_t s)
{
    SCHK(hipMemsetAsync(fB, 0, g.buf_bytes, s));
    SCHK(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    SCHK(init_populations(fA, g, s));
    SCHK(upload_particle(p, s));
    const SweepArgs sa = make_sweep_args(g);
    for (int64_t step = 0; step < n; ++step) {
        ParticleArgs<T> pa;
        fill_particle_args<T>(pa, g, seed, p, flags);
        pa.f = (const T*)fA;
        pa.trace = trace;
        pa.trace_cap = trace ? n : 0;
        pa.trace_start = 0;
        const int par = (int)(step & 1);
        pa.parity_in = par;
        pa.parity_out = par ^ 1;
        pa.check_zone = 0;
        // the hand-over words are written as in lbib_step's serial steps (nothing waits on them)
        pa.ready = p.d_count;
        pa.ready_value = (unsigned long long)step + 1;
        pa.zone_words = p.d_count + 2 + 2 * ((step + 1) & 3);
        pa.zone_tag = (uint32_t)((step + 1) & 0xffff);
        SCHK(launch_particle<T>(pa, s));
        SCHK(launch_sweep<T>((const T*)fA, (T*)fB, sa, p.d_desc, p.d_tile, g.pull, s, nullptr, nullptr,
                             reverse_sweep(g, step)));
        std::swap(fA, fB);
    }
    return LBIB_OK;
}

}  // namespace

}  // namespace lbib

using namespace lbib;

extern "C" lbib_status lbib_solve_static(const lbib_lattice_desc* lattice, const lbib_particle_desc* particle,
                                         const lbib_ligand_desc* ligands, int64_t n_steps, void* populations,
                                         int64_t* populations_bytes, lbib_particle_state* trace, uint8_t* bonds,
                                         void* hip_stream)
{
    try {
        if (!lattice || !particle || !ligands || !populations_bytes) return fail(LBIB_E_INVALID, "NULL argument");
        if (n_steps < 0 || n_steps > (int64_t(1) << 40)) return fail(LBIB_E_INVALID, "n_steps out of range");
        std::string msg;
        lbib_status v = check_lattice(*lattice, msg);
        if (v != LBIB_OK) return fail(v, msg);
        Particle p;
        v = prepare_particle(*lattice, *particle, p, msg);
        if (v != LBIB_OK) return fail(v, msg);
        v = check_ligands(*ligands, msg);
        if (v != LBIB_OK) return fail(v, msg);
        set_ligands(p, *ligands);
        LatticeGeom g = lattice_geom(*lattice);
        // the default layout of lbib_init
        g.pull = !g.interleaved && 2.0 * (double)g.buf_bytes > 512.0 * 1048576.0;
        const int64_t need_pop = 2 * (int64_t)align_up(g.buf_bytes);
        const size_t need_scratch = align_up(particle_block_bytes(p)) + kAlign;
        if (need_scratch > kStaticScratchBytes)
            return fail(LBIB_E_INVALID, "the particle needs " + std::to_string(need_scratch) +
                                            " bytes of device scratch; the static area holds " +
                                            std::to_string(kStaticScratchBytes));
        if (!populations) {
            *populations_bytes = need_pop;
            return LBIB_OK;
        }
        if (*populations_bytes < need_pop)
            return fail(LBIB_E_INVALID, "populations buffer of " + std::to_string(*populations_bytes) +
                                            " bytes; the lattice needs " + std::to_string(need_pop));
        if (((uintptr_t)populations & (kAlign - 1)) != 0)
            return fail(LBIB_E_INVALID, "populations must be aligned to 256 bytes");
        int dev = 0;
        SCHK(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices) return fail(LBIB_E_UNSUPPORTED, "device index beyond 63");
        std::lock_guard<std::mutex> lock(g_area[dev].mu);
        void* base = nullptr;
        SCHK(area_address(dev, &base));
        carve_particle(p, (char*)base);
        int32_t* flags = (int32_t*)((char*)base + align_up(particle_block_bytes(p)));
        char* fA = (char*)populations;
        char* fB = fA + align_up(g.buf_bytes);
        const hipStream_t s = (hipStream_t)hip_stream;
        switch (g.precision) {
            case LBIB_FP64: v = enqueue_solve<double>(g, lattice->seed, p, n_steps, fA, fB, trace, flags, s); break;
            case LBIB_FP32: v = enqueue_solve<float>(g, lattice->seed, p, n_steps, fA, fB, trace, flags, s); break;
            case LBIB_FP16: v = enqueue_solve<half_t>(g, lattice->seed, p, n_steps, fA, fB, trace, flags, s); break;
            case LBIB_BF16: v = enqueue_solve<bf16_t>(g, lattice->seed, p, n_steps, fA, fB, trace, flags, s); break;
            case LBIB_FP16_NEQ:
                v = enqueue_solve<half_neq_t>(g, lattice->seed, p, n_steps, fA, fB, trace, flags, s);
                break;
            default: v = enqueue_solve<bf16_neq_t>(g, lattice->seed, p, n_steps, fA, fB, trace, flags, s); break;
        }
        if (v != LBIB_OK) {
            (void)hipStreamSynchronize(s);
            return v;
        }
        if (bonds) SCHK(hipMemcpyAsync(bonds, p.d_bond, (size_t)p.nl, hipMemcpyDeviceToDevice, s));
        int32_t fl = 0;
        SCHK(hipMemcpyAsync(&fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
        // the host staging of the uploads and the lock are released only after the GPU is done
        SCHK(hipStreamSynchronize(s));
        if (fl) {
            std::string m = "numerical failure:";
            if (fl & FLAG_NONFINITE) m += " non-finite force/torque/velocity;";
            if (fl & FLAG_CONTACT) m += " particle touches the receptor wall (gap <= 0);";
            if (fl & FLAG_MLS) m += " singular MLS moment matrix;";
            if (fl & FLAG_TILE) m += " spread footprint exceeds the tile;";
            return fail(LBIB_E_NUMERIC, m);
        }
        return LBIB_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBIB_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(LBIB_E_INVALID, "unexpected error");
    }
}
