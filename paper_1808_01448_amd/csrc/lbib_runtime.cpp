// lbib_runtime.cpp -- host side of the LB-IB adhesion library: argument validation, unit
// conversion (Table 1 groups to lattice units), device allocation, the per-step launch
// sequence, read-outs, checkpoints and kernel timing.  Implements include/lbib.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "lbib.h"
#include "lbib_host.hpp"
#include "lbib_internal.hpp"

using namespace lbib;

namespace {

constexpr int kTimingPool = 8192;  // event pairs per kernel kind

constexpr int kKinds = 3;  // 0 lattice sweep, 1 particle phase, 2 second launch of the split phase

struct Timing {
    int32_t mask = 0;  // bit k: time kernel kind k
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
    hipStream_t stream3 = nullptr;  // its sweep: every CU but one (created at first use)
    bool masked = false;            // stream3 is CU-masked (the overlapped schedule needs it)
    int masked_dev = -1;            // the device whose masked-stream count it holds
    unsigned long long plaunches = 0;  // single-particle launches since lbib_init (hand-over counts)
    unsigned long long zdone_expected = 0;  // zone workgroups of the overlapped sweeps enqueued
    bool prev_overlapped = false;           // the last step enqueued ran overlapped
    hipEvent_t evA = nullptr, evB = nullptr, evC = nullptr;
    int overlap = 2;  // 0 serial, 1 overlapped, 2 chosen by lattice size, 3 split particle phase, 4 one-launch split phase
    int layout = 2;   // 0 push, 1 pull, 2 chosen by lattice size (at lbib_init)
    bool zone_valid = false;  // the zone slot of the next step holds its box
    int state = 0;  // 0 created, 1 running, 2 failed
    std::string err;
    LatticeGeom g;
    void* fA = nullptr;
    void* fB = nullptr;
    std::vector<Particle> parts;
    int32_t* d_flags = nullptr;
    // the flags word as of the end of the last lbib_step call, copied (stream-ordered) into
    // pinned host memory at that call's end, and the event that marks that end: lbib_sync and
    // the reads take the flags from there instead of a synchronous copy after their wait
    int32_t* h_flags = nullptr;
    bool h_flags_valid = false;
    hipEvent_t ev_end = nullptr;
    int64_t steps = 0;
    Timing timing;
    // split particle phase (several particles, or overlap mode 3): the two tile masks (by
    // step parity), every particle's box and tile, the particle arguments on the device
    unsigned long long* d_masks = nullptr;
    // hand-over counters of the split phase (they only grow): [0] the one-launch phase's grid
    // barrier (mode 4), [1] spread workgroups done, [2] loads workgroups done (the chained
    // schedule); the launches of each enqueued so far
    unsigned long long* d_bar = nullptr;
    uint64_t bar_launches = 0, spread_launches = 0, loads_launches = 0;
    int32_t mtx = 0;
    int64_t ntiles = 0;
    PartRef* d_refs = nullptr;
    void* d_args = nullptr;
    std::vector<unsigned char> h_args;  // host copy of the arguments (kept for the async upload)
    bool args_dirty = true;
    int32_t max_nl = 0;
    size_t lds_bytes = 0;
};

namespace {

// CU-masked streams held by live simulations, per device.  Each takes a hardware queue of its
// own, and the runtime does not refuse one too many but faults (a probe created 224 in one
// process, then the next creation crashed inside the runtime), so at most kMaxMaskedStreams
// simulations per device hold one; the others run the serial schedule (the same results).
constexpr int kMaxMaskedStreams = 8;
constexpr int kMaxDevices = 64;
std::mutex g_masked_mu;
int g_masked[kMaxDevices] = {};

bool take_masked_stream(int dev)
{
    std::lock_guard<std::mutex> lock(g_masked_mu);
    if (dev < 0 || dev >= kMaxDevices || g_masked[dev] >= kMaxMaskedStreams) return false;
    ++g_masked[dev];
    return true;
}

void give_masked_stream(int dev)
{
    std::lock_guard<std::mutex> lock(g_masked_mu);
    if (dev >= 0 && dev < kMaxDevices && g_masked[dev] > 0) --g_masked[dev];
}

// Whether every operation enqueued on the stream has completed (the query's not-ready status
// is cleared, so that it cannot be taken for a later launch's).
bool stream_idle(hipStream_t s)
{
    const hipError_t q = hipStreamQuery(s);
    if (q != hipSuccess) (void)hipGetLastError();
    return q == hipSuccess;
}

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

void free_all(lbib_sim* h)
{
    for (auto& p : h->parts) free_particle(p);
    if (h->fA) (void)hipFree(h->fA);
    if (h->fB) (void)hipFree(h->fB);
    h->fA = h->fB = nullptr;
    dfree(h->d_flags);
    if (h->h_flags) (void)hipHostFree(h->h_flags);
    h->h_flags = nullptr;
    h->h_flags_valid = false;
    if (h->ev_end) (void)hipEventDestroy(h->ev_end);
    h->ev_end = nullptr;
    dfree(h->d_masks);
    dfree(h->d_bar);
    dfree(h->d_refs);
    if (h->d_args) (void)hipFree(h->d_args);
    h->d_args = nullptr;
    for (int k = 0; k < kKinds; ++k) {
        for (auto e : h->timing.ev[k]) (void)hipEventDestroy(e);
        h->timing.ev[k].clear();
    }
    if (h->evA) (void)hipEventDestroy(h->evA);
    if (h->evB) (void)hipEventDestroy(h->evB);
    if (h->evC) (void)hipEventDestroy(h->evC);
    h->evA = h->evB = h->evC = nullptr;
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
    if (h->stream3) (void)hipStreamDestroy(h->stream3);
    h->stream2 = h->stream3 = nullptr;
    if (h->masked) give_masked_stream(h->masked_dev);
    h->masked = false;
}

template <typename T>
ParticleArgs<T> particle_args(lbib_sim* h, Particle& p)
{
    ParticleArgs<T> a;
    fill_particle_args<T>(a, h->g, h->desc.seed, p, h->d_flags);
    a.f = (const T*)h->fA;
    a.pid = (uint32_t)(&p - h->parts.data());  // the particle's index keys its bond draws
    a.refs = h->d_refs;
    a.mtx = h->mtx;
    a.nparts = (int32_t)h->parts.size();
    return a;
}

// Upload the arguments of the split particle phase (stream-ordered, from a host copy that
// stays alive until the next upload, which waits for the stream).
template <typename T>
lbib_status upload_split_args(lbib_sim* h)
{
    const size_t n = h->parts.size();
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->h_args.assign(n * sizeof(ParticleArgs<T>), 0);
    ParticleArgs<T>* a = (ParticleArgs<T>*)h->h_args.data();
    for (size_t k = 0; k < n; ++k) a[k] = particle_args<T>(h, h->parts[k]);
    HIPCHK(h, hipMemcpyAsync(h->d_args, a, h->h_args.size(), hipMemcpyHostToDevice, h->stream));
    h->args_dirty = false;
    return LBIB_OK;
}

SweepArgs sweep_args(lbib_sim* h) { return make_sweep_args(h->g); }

// Event pair that brackets the next launch of kernel `kind` (null when timing is off or the
// pool is used up).
struct EvPair {
    hipEvent_t t0 = nullptr, t1 = nullptr;
};

// `steps`: the steps the launch covers, counted as that many launches (the overlapped
// schedule's particle run).
EvPair timing_events(lbib_sim* h, int kind, int64_t steps = 1)
{
    Timing& t = h->timing;
    EvPair p;
    if (!(t.mask >> kind & 1) || t.used[kind] + 2 > t.ev[kind].size()) return p;
    p.t0 = t.ev[kind][t.used[kind]];
    p.t1 = t.ev[kind][t.used[kind] + 1];
    t.used[kind] += 2;
    t.launches[kind] += steps;
    return p;
}

// Longest run of steps one resident particle launch of the overlapped schedule covers; a
// longer call enqueues one such launch after another.
constexpr int64_t kRunSteps = 1024;

// The overlapped schedule's sweep stream: a CU mask that leaves one CU out of the sweep, a
// CU its workgroups can never hold while they wait on the device for the particle's.  (A
// one-workgroup launch goes to the XCD and shader engine its queue chooses, not to that CU:
// measured, the particle's workgroup used eight CUs of one shader engine and never the free
// one, for any one of the mask bits tried.  It starts once enough of a CU is free, which a
// dispatching sweep refills as fast as its workgroups retire: a particle launch per step that
// misses a sweep's drain runs after the next one's, and the step takes 59 instead of 46 us at
// 4096 x 1024 until the call ends, which is why mode 2 keeps one particle launch resident over
// a call's steps.  Leaving one CU of every XCD out measured 3 % slower.)
// Created at the first overlapped step (each masked stream holds a hardware queue); without
// CU masking the overlapped schedule stays off.
hipError_t ensure_sweep_stream(lbib_sim* h)
{
    if (h->stream3) return hipSuccess;
    hipError_t e = hipEventCreateWithFlags(&h->evC, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    int dev = 0;
    hipDeviceProp_t prop;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e == hipSuccess && prop.multiProcessorCount > 64 && take_masked_stream(dev)) {
        const int n = prop.multiProcessorCount;
        std::vector<uint32_t> mask((size_t)(n + 31) / 32, 0u);
        for (int cu = 1; cu < n; ++cu) mask[cu / 32] |= 1u << (cu % 32);
        if (hipExtStreamCreateWithCUMask(&h->stream3, (uint32_t)mask.size(), mask.data()) == hipSuccess) {
            h->masked = true;
            h->masked_dev = dev;
            return hipSuccess;
        }
        give_masked_stream(dev);
        (void)hipGetLastError();
    }
    // no CU masking (or every masked stream of the device taken): the overlapped schedule
    // stays off (the stream marks the attempt)
    return hipStreamCreateWithFlags(&h->stream3, hipStreamNonBlocking);
}

// One time step is the particle phase then the lattice sweep.  Serial schedule: both on the
// caller's stream.  Overlapped schedule (when the previous step has predicted this step's
// box): the particle phase runs on the second stream while the caller's stream sweeps the
// lattice on a third, with no event between the two chains but the particle's wait for the
// previous sweep: the sweep waits on the device for the previous particle launch, and the
// tiles of the predicted box, which need the spread force, go to workgroups at the head of
// its grid, which wait for the force to be published (HandoverArgs).  Both schedules compute
// every node with the same arithmetic.
template <typename T>
lbib_status enqueue_steps(lbib_sim* h, int64_t n)
{
    const SweepArgs sa = sweep_args(h);
    bool joined = true;
    // a caller's stream with nothing pending needs no join before the other streams start (no
    // event and cross-stream wait at the call's start: ~20 us of a short call); anything this
    // call enqueues on it clears this
    bool idle = stream_idle(h->stream);
    int64_t run_left = 0;  // steps still covered by the resident particle launch already enqueued
    h->h_flags_valid = false;  // until this call's copy is enqueued
    const bool split = h->parts.size() > 1 || (h->overlap == 3 && !h->parts.empty());
    if (split && h->args_dirty) {
        lbib_status st = upload_split_args<T>(h);
        if (st != LBIB_OK) return st;
    }
    for (int64_t s = 0; s < n; ++s) {
        const T* fin = (const T*)h->fA;
        T* fout = (T*)h->fB;
        if (split) {
            // every particle spreads and marks the tile mask, then every particle evaluates its
            // loads (seeing all spread forces) and moves, then the lattice is swept
            const int par = (int)(h->steps & 1);
            unsigned long long* mcur = h->d_masks + par * h->ntiles;
            unsigned long long* mnext = h->d_masks + (par ^ 1) * h->ntiles;
            const int32_t np = (int32_t)h->parts.size();
            const ParticleArgs<T>* args = (const ParticleArgs<T>*)h->d_args;
            // chained schedule (mode 1): the loads launch of step n runs on the second
            // stream beside the sweep of step n; the two streams hand over on the device.  The
            // loads launch starts once every spread workgroup of step n has counted in; the
            // spread launch of step n+1 (after the sweep of step n on the caller's stream)
            // once every loads workgroup of step n has (it rewrites the force lists those read,
            // and the particle state they write), so the sweep of step n+1, which overwrites
            // the populations the loads of step n read, follows it.  No launch waits for a
            // later one, and no workgroup waits for another of its own launch.
            // Modes 2 (the default) and 4: both halves as one launch whose workgroups claim the
            // particles and meet between the halves (no second launch, and each workgroup
            // stages its supports once); a workgroup that finds a particle unclaimed there does
            // its work itself, so no co-residency is assumed.  Mode 5: the same launch on one
            // workgroup, which then takes that path every step.  Modes 0 and 3: the two
            // launches and the sweep in order on the caller's stream.
            const bool chain = h->overlap == 1;
            const bool one_launch = h->overlap == 2 || h->overlap == 4 || h->overlap == 5;
            if (chain && joined) {  // the second stream starts after the caller's work
                if (!idle) {
                    HIPCHK(h, hipEventRecord(h->evA, h->stream));
                    HIPCHK(h, hipStreamWaitEvent(h->stream2, h->evA, 0));
                }
                joined = false;
            }
            idle = false;  // the launches below go (at least in part) to the caller's stream
            if (one_launch) {
                const EvPair e1 = timing_events(h, 1);
                if (e1.t0) HIPCHK(h, hipEventRecord(e1.t0, h->stream));
                const unsigned long long target = (unsigned long long)(h->bar_launches + 1) * (unsigned long long)np;
                HIPCHK(h, launch_particle_fused<T>(args, np, h->overlap == 5 ? 1 : np, fin, mcur, h->max_nl,
                                                   h->lds_bytes, h->d_bar, target, h->stream));
                h->bar_launches += 1;
                if (e1.t1) HIPCHK(h, hipEventRecord(e1.t1, h->stream));
            } else {
                SplitChain c1, c2;
                if (chain) {
                    c1.wait = h->d_bar + 2;
                    c1.wait_target = (unsigned long long)np * h->loads_launches;
                    c1.done = h->d_bar + 1;
                    c2.wait = h->d_bar + 1;
                    c2.wait_target = (unsigned long long)np * (h->spread_launches + 1);
                    c2.done = h->d_bar + 2;
                }
                const EvPair e1 = timing_events(h, 1);
                HIPCHK(h, launch_particle_split<T>(args, np, fin, mcur, 1, h->max_nl, h->lds_bytes, h->stream, e1.t0,
                                                   e1.t1, c1));
                const EvPair e2 = timing_events(h, 2);
                HIPCHK(h, launch_particle_split<T>(args, np, fin, mcur, 2, h->max_nl, h->lds_bytes,
                                                   chain ? h->stream2 : h->stream, e2.t0, e2.t1, c2));
                h->spread_launches += 1;
                h->loads_launches += 1;
            }
            const EvPair e0 = timing_events(h, 0);
            HIPCHK(h, launch_sweep_multi<T>(fin, fout, sa, mcur, mnext, h->d_refs, h->g.pull, h->stream, e0.t0, e0.t1));
            h->zone_valid = false;
        } else if (h->parts.empty()) {
            idle = false;
            const EvPair e0 = timing_events(h, 0);
            HIPCHK(h, launch_sweep<T>(fin, fout, sa, nullptr, nullptr, h->g.pull, h->stream, e0.t0, e0.t1,
                                      reverse_sweep(h->g, h->steps)));
        } else {
            Particle& p = h->parts[0];
            ParticleArgs<T> pa = particle_args<T>(h, p);
            const int par = (int)(h->steps & 1);
            pa.parity_in = par;
            pa.parity_out = par ^ 1;
            // hand-over (HandoverArgs): this launch publishes its force as count launches + 1
            // and its box prediction with that tag in slot (step + 1) mod 4; the previous
            // launch's carries launches, in slot step mod 4
            const unsigned long long prev = h->plaunches;
            pa.ready = p.d_count;
            pa.ready_value = prev + 1;
            pa.zone_words = p.d_count + 2 + 2 * ((h->steps + 1) & 3);
            pa.zone_tag = (uint32_t)((prev + 1) & 0xffffu);
            h->plaunches = prev + 1;
            // the overlapped schedule is the faster one at every size measured, from 256 x 64
            // (20.1 against 21.9 us per step: the sweep hides behind the particle phase) to
            // 8192 x 4096 (the particle phase hides behind the sweep).  It needs the CU-masked
            // sweep stream: workgroups of the sweep and the particle's wait for each other on
            // the device, and the particle must always find a CU.
            bool overlap = h->overlap == 1 || h->overlap == 2;
            if (h->desc.ny >= (1 << 23)) overlap = false;  // the packed tiles (zone_pack)
            if (overlap && h->zone_valid) HIPCHK(h, ensure_sweep_stream(h));
            if (!h->masked) overlap = false;
            if (!overlap || !h->zone_valid) {
                if (!joined) {  // the previous step ran overlapped
                    HIPCHK(h, hipEventRecord(h->evA, h->stream3));
                    HIPCHK(h, hipEventRecord(h->evB, h->stream2));
                    HIPCHK(h, hipStreamWaitEvent(h->stream, h->evA, 0));
                    HIPCHK(h, hipStreamWaitEvent(h->stream, h->evB, 0));
                    joined = true;
                }
                if (run_left != 0) return fail(h, LBIB_E_STATE, "lbib_step: a serial step inside a resident particle run");
                pa.check_zone = 0;
                idle = false;
                const EvPair e1 = timing_events(h, 1);
                HIPCHK(h, launch_particle<T>(pa, h->stream, e1.t0, e1.t1));
                const EvPair e0 = timing_events(h, 0);
                HIPCHK(h, launch_sweep<T>(fin, fout, sa, p.d_desc, p.d_tile, h->g.pull, h->stream, e0.t0, e0.t1,
                                          reverse_sweep(h->g, h->steps)));
                h->zone_valid = true;
                h->prev_overlapped = false;
            } else {
                if (joined && !idle) {  // both chains start after the caller's work
                    HIPCHK(h, hipEventRecord(h->evC, h->stream));
                    HIPCHK(h, hipStreamWaitEvent(h->stream2, h->evC, 0));
                    HIPCHK(h, hipStreamWaitEvent(h->stream3, h->evC, 0));
                }
                // the particle launch waits on the device for the previous sweep's zone
                // workgroups; the sweep, for the previous particle launch's box and, in its
                // zone workgroups, for this one's force: no event between the two chains
                pa.check_zone = 1;
                pa.zdone = p.d_count + 1;
                pa.zdone_target = h->zdone_expected;
                pa.check_prev = h->prev_overlapped ? 1 : 0;
                const int nzone = zone_workgroups(p, h->g.pull);
                if (h->overlap == 1) {  // a launch per step
                    const EvPair e1 = timing_events(h, 1);
                    HIPCHK(h, launch_particle<T>(pa, h->stream2, e1.t0, e1.t1));
                } else {
                    // mode 2: one launch for this step and the call's later ones (every later
                    // step of the call is overlapped too), its workgroup resident between them
                    if (run_left == 0) {
                        const int64_t len = std::min<int64_t>(n - s, kRunSteps);
                        const ParticleRun<T> run{fin, (const T*)h->fB, p.d_count + 2, h->steps, (int32_t)len, nzone};
                        const EvPair e1 = timing_events(h, 1, len);
                        HIPCHK(h, launch_particle_run<T>(pa, run, h->stream2, e1.t0, e1.t1));
                        run_left = len;
                    }
                    --run_left;
                }
                const HandoverArgs ha{p.d_count + 2 + 2 * (h->steps & 3), (uint32_t)(prev & 0xffffu), p.d_desc, p.d_tile,
                                      p.d_count, prev + 1, p.d_count + 1, h->d_flags, nzone};
                const EvPair e0 = timing_events(h, 0);
                HIPCHK(h, launch_sweep_overlap<T>(fin, fout, sa, ha, h->g.pull, h->stream3, e0.t0, e0.t1,
                                                  reverse_sweep(h->g, h->steps)));
                h->zdone_expected += (unsigned long long)nzone;
                h->prev_overlapped = true;
                joined = false;
            }
        }
        std::swap(h->fA, h->fB);
        h->steps += 1;
    }
    if (!joined) {
        // everything enqueued is ordered before later work on the caller's stream: the sweep
        // chain of one overlapped particle, and the second stream (its particle chain, or the
        // loads launches of the chained split phase)
        if (h->prev_overlapped && !split) {
            HIPCHK(h, hipEventRecord(h->evA, h->stream3));
            HIPCHK(h, hipStreamWaitEvent(h->stream, h->evA, 0));
        }
        HIPCHK(h, hipEventRecord(h->evB, h->stream2));
        HIPCHK(h, hipStreamWaitEvent(h->stream, h->evB, 0));
    }
    if (n > 0) {
        HIPCHK(h, hipMemcpyAsync(h->h_flags, h->d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipEventRecord(h->ev_end, h->stream));
        h->h_flags_valid = true;
    }
    return LBIB_OK;
}

// Callers have synchronised the handle's stream, so the copy of the last lbib_step call has
// landed.
lbib_status check_flags(lbib_sim* h)
{
    int32_t fl = 0;
    if (h->h_flags_valid)
        fl = *(volatile int32_t*)h->h_flags;
    else
        HIPCHK(h, hipMemcpy(&fl, h->d_flags, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl) {
        h->state = 2;
        std::string m = "numerical failure:";
        if (fl & FLAG_NONFINITE) m += " non-finite force/torque/velocity;";
        if (fl & FLAG_CONTACT) m += " particle touches the receptor wall (gap <= 0);";
        if (fl & FLAG_MLS) m += " singular MLS moment matrix;";
        if (fl & FLAG_TILE) m += " spread footprint exceeds the tile;";
        if (fl & FLAG_SYNC) m += " device-side wait timed out;";
        return fail(h, LBIB_E_NUMERIC, m);
    }
    return LBIB_OK;
}

// Waits for the handle's stream.  The end of the last lbib_step call is polled for up to
// 2 ms first (a blocking wait's wake-up costs tens of microseconds, a large share of a short
// call); longer waits block.
lbib_status sync_check(lbib_sim* h)
{
    if (h->h_flags_valid) {
        const auto t0 = std::chrono::steady_clock::now();
        hipError_t q;
        while ((q = hipEventQuery(h->ev_end)) == hipErrorNotReady)
            if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000)) break;
        if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(h, q, "hipEventQuery");
    }
    if (!stream_idle(h->stream)) HIPCHK(h, hipStreamSynchronize(h->stream));
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
    HIPCHK(h, download_populations(h->fA, h->g, f));
    return LBIB_OK;
}

struct BlobHeader {
    char magic[8];
    int32_t version, nx, ny, precision, n_particles, nl;
    int32_t layout;  // blob_layout: bit 0 pull, bit 1 row-interleaved buffers
    int64_t steps, pop_bytes;
};

int32_t blob_layout(const LatticeGeom& g) { return (g.pull ? 1 : 0) | (g.interleaved ? 2 : 0); }

size_t blob_size(lbib_sim* h)
{
    size_t s = sizeof(BlobHeader) + h->g.buf_bytes;
    for (auto& p : h->parts) s += sizeof(DevParticle) + (size_t)p.nl;
    return s;
}

}  // namespace

void lbib::set_null_error(const std::string& msg) { g_null_err = msg; }

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
        std::string msg;
        const lbib_status v = check_lattice(*d, msg);
        if (v != LBIB_OK) return fail(nullptr, v, "lbib_create: " + msg);
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
        h->g = lattice_geom(*d);
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
        if (h->parts.size() >= 64) return fail(h, LBIB_E_UNSUPPORTED, "lbib_particle_add: at most 64 particles");
        Particle p;
        std::string msg;
        const lbib_status v = prepare_particle(h->desc, *d, p, msg);
        if (v != LBIB_OK) return fail(h, v, "lbib_particle_add: " + msg);
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
    std::string msg;
    const lbib_status v = check_ligands(*d, msg);
    if (v != LBIB_OK) return fail(h, v, "lbib_ligands_set: " + msg);
    try {
        set_ligands(*p, *d);
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_ligands_set: host allocation failed");
    }
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
    const size_t bytes = h->g.buf_bytes;
    // in row-interleaved buffers the push update is the faster one at the sizes measured (up
    // to 2.4 GB per buffer, every storage); in population planes (rows too long for a 32-bit
    // pitch) its shifted stores are cheap only while both buffers fit the 256 MB MALL beside
    // the rest of the working set, and far above it the pull update's aligned stores win
    h->g.pull = h->layout == 1 || (h->layout == 2 && !h->g.interleaved && 2.0 * bytes > 512.0 * 1048576.0);
    hipError_t e;
    if ((e = hipMalloc(&h->fA, bytes)) != hipSuccess || (e = hipMalloc(&h->fB, bytes)) != hipSuccess ||
        (e = dalloc(&h->d_flags, 1)) != hipSuccess) {
        free_all(h);
        return fail(h, e == hipErrorOutOfMemory ? LBIB_E_NOMEM : LBIB_E_DEVICE,
                    std::string("lbib_init: device allocation: ") + hipGetErrorString(e));
    }
    for (auto& p : h->parts) {
        if ((e = alloc_particle(p)) != hipSuccess) {
            free_all(h);
            return fail(h, e == hipErrorOutOfMemory ? LBIB_E_NOMEM : LBIB_E_DEVICE,
                        std::string("lbib_init: device allocation: ") + hipGetErrorString(e));
        }
    }
    auto bail = [&](hipError_t err, const char* what) {
        free_all(h);
        return hip_fail(h, err, what);
    };
    if ((e = hipMemsetAsync(h->fB, 0, bytes, h->stream)) != hipSuccess) return bail(e, "hipMemset");
    if ((e = hipMemsetAsync(h->d_flags, 0, sizeof(int32_t), h->stream)) != hipSuccess) return bail(e, "hipMemset");
    if ((e = hipHostMalloc((void**)&h->h_flags, sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->ev_end, hipEventDisableTiming)) != hipSuccess)
        return bail(e, "lbib_init: pinned flags");
    *h->h_flags = 0;
    h->h_flags_valid = false;
    if ((e = init_populations(h->fA, h->g, h->stream)) != hipSuccess) return bail(e, "init kernel");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return bail(e, "lbib_init: sync");
    for (auto& p : h->parts)
        if ((e = upload_particle(p, h->stream)) != hipSuccess) return bail(e, "lbib_init: upload");
    if (!h->parts.empty()) {
        // tile masks, particle references and arguments of the split particle phase
        h->mtx = (h->desc.nx + 63) / 64;
        h->ntiles = (int64_t)h->mtx * ((h->desc.ny + 3) / 4);
        const size_t np = h->parts.size();
        std::vector<PartRef> refs(np);
        for (size_t k = 0; k < np; ++k) {
            refs[k] = PartRef{h->parts[k].d_desc, h->parts[k].d_tile, h->parts[k].d_ring};
            const Particle& p = h->parts[k];
            h->max_nl = std::max(h->max_nl, p.nl);
            h->lds_bytes = std::max(h->lds_bytes, particle_launch_lds(p.box_cap));
        }
        const size_t args_bytes = np * std::max(sizeof(ParticleArgs<double>), sizeof(ParticleArgs<float>));
        // monotonic counters: [0] spreads of the one-launch phase, [1] [2] the chained
        // schedule's hand-over, [3] the one-launch phase's claims, then one claim word per
        // particle (up to 64)
        constexpr size_t kCounters = 4 + 64;
        h->bar_launches = h->spread_launches = h->loads_launches = 0;
        if ((e = dalloc(&h->d_bar, kCounters)) != hipSuccess ||
            (e = hipMemsetAsync(h->d_bar, 0, kCounters * sizeof(unsigned long long), h->stream)) != hipSuccess)
            return bail(e, "lbib_init: hand-over counters");
        if ((e = dalloc(&h->d_masks, (size_t)(2 * h->ntiles))) != hipSuccess ||
            (e = dalloc(&h->d_refs, np)) != hipSuccess || (e = hipMalloc(&h->d_args, args_bytes)) != hipSuccess)
            return bail(e, "lbib_init: device allocation");
        if ((e = hipMemsetAsync(h->d_masks, 0, (size_t)(2 * h->ntiles) * 8, h->stream)) != hipSuccess ||
            (e = hipMemcpy(h->d_refs, refs.data(), np * sizeof(PartRef), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "lbib_init: upload");
        h->args_dirty = true;
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
    switch (h->g.precision) {
        case LBIB_FP64: return enqueue_steps<double>(h, n);
        case LBIB_FP32: return enqueue_steps<float>(h, n);
        case LBIB_FP16: return enqueue_steps<half_t>(h, n);
        case LBIB_BF16: return enqueue_steps<bf16_t>(h, n);
        case LBIB_FP16_NEQ: return enqueue_steps<half_neq_t>(h, n);
        default: return enqueue_steps<bf16_neq_t>(h, n);
    }
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
    const int64_t need = (which == 3 ? 9 : 1) * (int64_t)h->desc.nx * h->desc.ny;
    if (capacity < need) return fail(h, LBIB_E_INVALID, "lbib_read_field: capacity must be >= " + std::to_string(need));
    try {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        std::vector<double> f;
        lbib_status s = download_f(h, f);
        if (s != LBIB_OK) return s;
        field_from_populations(f, h->g, which, out);
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
    if (count != (int64_t)9 * h->desc.nx * h->desc.ny)
        return fail(h, LBIB_E_INVALID, "lbib_write_populations: count must be 9 nx ny");
    try {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        HIPCHK(h, upload_populations(h->fA, h->g, f));
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
    h->args_dirty = true;
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
    std::memcpy(hd.magic, "LBIBCKP3", 8);
    hd.version = LBIB_ABI_VERSION;
    hd.nx = h->desc.nx;
    hd.ny = h->desc.ny;
    hd.precision = h->desc.precision;
    hd.n_particles = (int32_t)h->parts.size();
    hd.nl = h->parts.empty() ? 0 : h->parts[0].nl;
    hd.layout = blob_layout(h->g);
    hd.steps = h->steps;
    hd.pop_bytes = (int64_t)h->g.buf_bytes;
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
    if (std::memcmp(hd.magic, "LBIBCKP3", 8) != 0 || hd.version != LBIB_ABI_VERSION || hd.nx != h->desc.nx ||
        hd.layout != blob_layout(h->g) ||
        hd.ny != h->desc.ny || hd.precision != h->desc.precision || hd.n_particles != (int32_t)h->parts.size() ||
        (hd.n_particles && hd.nl != h->parts[0].nl) || hd.pop_bytes != (int64_t)h->g.buf_bytes)
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
        h->args_dirty = true;
    }
    const int32_t zero = 0;
    HIPCHK(h, hipMemcpy(h->d_flags, &zero, sizeof(zero), hipMemcpyHostToDevice));
    h->h_flags_valid = false;
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
    t.mask = enable & 7;
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
    if (mode < 0 || mode > 5) return fail(h, LBIB_E_INVALID, "lbib_set_overlap: mode must be 0 to 5");
    h->overlap = mode;
    return LBIB_OK;
}

lbib_status lbib_set_layout(lbib_handle h, int32_t mode)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_set_layout: NULL handle");
    if (mode < 0 || mode > 2) return fail(h, LBIB_E_INVALID, "lbib_set_layout: mode must be 0, 1 or 2");
    if (h->state != 0) return fail(h, LBIB_E_STATE, "lbib_set_layout: must precede lbib_init");
    h->layout = mode;
    return LBIB_OK;
}

lbib_status lbib_get_layout(lbib_handle h, int32_t* pull)
{
    if (!h || !pull) return fail(h, LBIB_E_INVALID, "lbib_get_layout: NULL argument");
    if (h->state == 0) return fail(h, LBIB_E_STATE, "lbib_get_layout: the layout is chosen by lbib_init");
    *pull = h->g.pull ? 1 : 0;
    return LBIB_OK;
}

lbib_status lbib_bytes_per_update(lbib_handle h, int64_t* bytes)
{
    if (!h || !bytes) return fail(h, LBIB_E_INVALID, "lbib_bytes_per_update: NULL argument");
    *bytes = (int64_t)h->g.upd_bytes;
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
