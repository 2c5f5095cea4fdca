// lbib_pool.cpp -- many independent LB-IB adhesion simulations stepped together: one
// particle-phase launch (one workgroup per member) and one lattice-sweep launch (the tiles
// of every member) per time step, instead of two launches and two launch gaps per member.
// Members differ in lattice size, particle, ligands and seed, join and leave between
// calls, and each runs its own number of steps; every member's result is bit-identical to
// the same simulation run alone through lbib_create / lbib_step (serial schedule), since
// both run the same device functions on the same data.  Implements the pool part of
// include/lbib.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "lbib.h"
#include "lbib_host.hpp"
#include "lbib_internal.hpp"

using namespace lbib;

namespace {

constexpr int kPoolTimingPool = 8192;  // event pairs per kernel kind

// First-fit sub-allocator over one device allocation made when the pool is created, so a
// member joins and leaves without a device allocation or free (each of which would wait for
// the whole device).  Blocks are multiples of 256 bytes; freed blocks merge with free
// neighbours.
class Arena {
  public:
    hipError_t init(size_t bytes)
    {
        size_ = align_up(bytes);
        hipError_t e = hipMalloc((void**)&base_, size_);
        if (e != hipSuccess) {
            base_ = nullptr;
            size_ = 0;
            return e;
        }
        free_[0] = size_;
        return hipSuccess;
    }
    void release()
    {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        size_ = 0;
        free_.clear();
    }
    // nullptr when no free block is large enough
    char* alloc(size_t bytes)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            return base_ + off;
        }
        return nullptr;
    }
    void free(char* p, size_t bytes)
    {
        size_t off = (size_t)(p - base_), len = align_up(bytes);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }

  private:
    char* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Member {
    int32_t slot = -1;
    int32_t lane = -1;  // index into the pool-wide state and flag arrays
    lbib_lattice_desc lat{};
    LatticeGeom g;
    Particle p;
    void* fA = nullptr;
    void* fB = nullptr;
    char* block = nullptr;  // the member's arena block: fA, fB, then the particle's buffers
    int64_t target = 0;
    int64_t bytes = 0;
    int32_t state = LBIB_POOL_RUNNING;
    int64_t steps_done = 0;  // as of the last poll
    bool reported = false;   // finished / failed already returned by a poll
};

}  // namespace

struct lbib_pool {
    int32_t precision = LBIB_FP32;
    size_t elem = 4;
    int64_t budget = 0, in_use = 0;
    int32_t max_members = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::map<int32_t, std::unique_ptr<Member>> members;
    int32_t next_slot = 0;
    std::vector<int32_t> free_lanes;
    // pool-wide device arrays, one entry per lane
    DevParticle* d_st = nullptr;
    int32_t* d_flags = nullptr;
    Arena arena;  // members' device memory
    // host snapshot of every lane's particle state and flags, valid while nothing has been
    // enqueued since it was taken
    std::vector<DevParticle> st_cache;
    std::vector<int32_t> fl_cache;
    bool cache_valid = false;
    // launch tables (rebuilt when the set of running members changes)
    bool dirty = true;
    void* d_args = nullptr;
    size_t args_cap = 0;
    int32_t* d_active = nullptr;
    size_t active_cap = 0;
    void* d_sims = nullptr;
    size_t sims_cap = 0;
    int2* d_table = nullptr;
    size_t table_cap = 0;
    TileDesc* d_ctl = nullptr;  // per running member: its box of the step and the step parity
    size_t ctl_cap = 0;
    int32_t n_active = 0, n_blocks = 0, max_nl = 0;
    size_t lds_bytes = 0;
    PoolSweepConfig cfg{256, 4};
    // optional replay of graph_steps steps as one HIP graph (rebuilt with the tables)
    int32_t graph_steps = 0;
    hipGraphExec_t graph = nullptr;
    int64_t pool_steps = 0;
    // kernel timing: kind 0 sweep, 1 particle phase
    bool timing = false;
    std::vector<hipEvent_t> ev[2];
    size_t ev_used[2] = {0, 0};
    int64_t launches[2] = {0, 0};
};

namespace {

thread_local std::string g_pool_null_err;

lbib_status fail(lbib_pool* h, lbib_status s, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_pool_null_err = msg;
    return s;
}

lbib_status hip_fail(lbib_pool* h, hipError_t e, const std::string& what)
{
    return fail(h, e == hipErrorOutOfMemory ? LBIB_E_NOMEM : LBIB_E_DEVICE, what + ": " + hipGetErrorString(e));
}

#define PCHK(h, call)                                               \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call);      \
    } while (0)

// The stream must be idle (no enqueued step may still use the block).
void free_member(lbib_pool* h, Member& m)
{
    free_particle(m.p);  // the block is the arena's; only an optional trace buffer is freed
    if (m.block) h->arena.free(m.block, (size_t)m.bytes);
    m.block = nullptr;
    m.fA = m.fB = nullptr;
}

template <typename T>
void ensure(T*& d, size_t& cap, size_t need, hipError_t& e)
{
    if (e != hipSuccess || need <= cap) return;
    size_t c = std::max<size_t>(need, cap * 2);
    if (d) (void)hipFree((void*)d);
    d = nullptr;
    cap = 0;
    e = hipMalloc((void**)&d, c * sizeof(T));
    if (e == hipSuccess) cap = c;
}

// Rebuild the launch tables from the running members (the stream is idle when called).
// Members with the most markers come first so the longest particle phases start first.
template <typename T>
lbib_status rebuild(lbib_pool* h)
{
    std::vector<Member*> run;
    for (auto& kv : h->members)
        if (kv.second->state == LBIB_POOL_RUNNING) run.push_back(kv.second.get());
    std::stable_sort(run.begin(), run.end(), [](const Member* a, const Member* b) { return a->p.nl > b->p.nl; });
    std::vector<ParticleArgs<T>> args(run.size());
    std::vector<int32_t> active(run.size());
    std::vector<PoolSweep<T>> sims(run.size());
    std::vector<int2> table;
    int32_t max_nl = 0;
    size_t lds_bytes = 0;
    for (size_t k = 0; k < run.size(); ++k) {
        Member& m = *run[k];
        ParticleArgs<T>& a = args[k];
        fill_particle_args<T>(a, m.g, m.lat.seed, m.p, h->d_flags + m.lane);
        a.f = (const T*)m.fA;
        a.fB = (const T*)m.fB;
        a.target_steps = m.target;
        a.check_zone = 0;
        a.parity_in = 0;
        a.parity_out = 1;
        active[k] = (int32_t)k;
        max_nl = std::max(max_nl, m.p.nl);
        lds_bytes = std::max(lds_bytes, particle_launch_lds(m.p.box_cap));
        PoolSweep<T>& s = sims[k];
        s = PoolSweep<T>{};
        s.a = make_sweep_args(m.g);
        s.fA = (T*)m.fA;
        s.fB = (T*)m.fB;
        s.tile = m.p.d_tile;
        const int by = 256 / h->cfg.bx;
        const int gx = (m.g.nx + h->cfg.bx - 1) / h->cfg.bx;
        s.gx = make_fastdiv((uint32_t)gx);
        s.ntiles = gx * ((m.g.ny + by - 1) / by);
        if ((int64_t)table.size() + s.ntiles / h->cfg.tpb + 1 > 0x7fffffff)
            return fail(h, LBIB_E_INVALID, "pool: more than 2^31 sweep blocks");
        for (int32_t t = 0; t < s.ntiles; t += h->cfg.tpb) table.push_back(make_int2((int)k, t));
    }
    hipError_t e = hipSuccess;
    ParticleArgs<T>* dargs = (ParticleArgs<T>*)h->d_args;
    PoolSweep<T>* dsims = (PoolSweep<T>*)h->d_sims;
    ensure(dargs, h->args_cap, args.size(), e);
    h->d_args = dargs;
    ensure(h->d_active, h->active_cap, active.size(), e);
    ensure(dsims, h->sims_cap, sims.size(), e);
    h->d_sims = dsims;
    ensure(h->d_table, h->table_cap, table.size(), e);
    ensure(h->d_ctl, h->ctl_cap, run.size(), e);
    if (e != hipSuccess) return hip_fail(h, e, "pool: table allocation");
    if (!run.empty()) {
        PCHK(h, hipMemcpy(h->d_args, args.data(), args.size() * sizeof(ParticleArgs<T>), hipMemcpyHostToDevice));
        PCHK(h, hipMemcpy(h->d_active, active.data(), active.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        PCHK(h, hipMemcpy(h->d_sims, sims.data(), sims.size() * sizeof(PoolSweep<T>), hipMemcpyHostToDevice));
        PCHK(h, hipMemcpy(h->d_table, table.data(), table.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    h->n_active = (int32_t)run.size();
    h->n_blocks = (int32_t)table.size();
    h->max_nl = max_nl;
    h->lds_bytes = lds_bytes;
    h->dirty = false;
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    return LBIB_OK;
}

struct EvPair {
    hipEvent_t t0 = nullptr, t1 = nullptr;
};

EvPair next_events(lbib_pool* h, int kind)
{
    EvPair p;
    if (!h->timing || h->ev_used[kind] + 2 > h->ev[kind].size()) return p;
    p.t0 = h->ev[kind][h->ev_used[kind]];
    p.t1 = h->ev[kind][h->ev_used[kind] + 1];
    h->ev_used[kind] += 2;
    h->launches[kind] += 1;
    return p;
}

template <typename T>
hipError_t launch_step(lbib_pool* h, EvPair e1, EvPair e0)
{
    hipError_t e = launch_pool_particle<T>((const ParticleArgs<T>*)h->d_args, h->d_active, h->d_ctl, h->n_active,
                                           h->max_nl, h->lds_bytes, h->stream, e1.t0, e1.t1);
    if (e != hipSuccess) return e;
    return launch_pool_sweep<T>((const PoolSweep<T>*)h->d_sims, h->d_ctl, h->d_table, h->n_blocks, h->cfg, h->stream,
                                e0.t0, e0.t1);
}

// Capture graph_steps steps of direct launches into one executable graph.
template <typename T>
lbib_status build_graph(lbib_pool* h)
{
    hipGraph_t g = nullptr;
    PCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < h->graph_steps && e == hipSuccess; ++k) e = launch_step<T>(h, EvPair{}, EvPair{});
    hipError_t e2 = hipStreamEndCapture(h->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(h, e != hipSuccess ? e : e2, "pool: graph capture");
    }
    e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph = nullptr;
        return hip_fail(h, e, "pool: graph instantiation");
    }
    return LBIB_OK;
}

template <typename T>
lbib_status enqueue(lbib_pool* h, int64_t n)
{
    if (h->dirty) {
        PCHK(h, hipStreamSynchronize(h->stream));  // in-flight steps may still read the tables
        lbib_status s = rebuild<T>(h);
        if (s != LBIB_OK) return s;
    }
    if (h->n_active == 0) return LBIB_OK;
    h->cache_valid = false;
    int64_t k = 0;
    if (h->graph_steps > 0 && !h->timing && n >= h->graph_steps) {
        if (!h->graph) {
            lbib_status s = build_graph<T>(h);
            if (s != LBIB_OK) return s;
        }
        for (; k + h->graph_steps <= n; k += h->graph_steps) PCHK(h, hipGraphLaunch(h->graph, h->stream));
    }
    for (; k < n; ++k) {
        const EvPair e1 = next_events(h, 1);
        const EvPair e0 = next_events(h, 0);
        PCHK(h, launch_step<T>(h, e1, e0));
    }
    h->pool_steps += n;
    return LBIB_OK;
}

bool valid_config(int32_t bx, int32_t tpb)
{
    return (bx == 64 || bx == 128 || bx == 256) && (tpb == 1 || tpb == 2 || tpb == 4 || tpb == 8);
}

Member* get_member(lbib_pool* h, int32_t slot)
{
    auto it = h->members.find(slot);
    return it == h->members.end() ? nullptr : it->second.get();
}

// Synchronise and refresh every member's step count and state from the device (a no-op
// while the last snapshot is still current).
lbib_status refresh(lbib_pool* h)
{
    if (h->cache_valid) return LBIB_OK;
    PCHK(h, hipStreamSynchronize(h->stream));
    int32_t top = 0;
    for (auto& kv : h->members) top = std::max(top, kv.second->lane + 1);
    std::vector<DevParticle>& st = h->st_cache;
    std::vector<int32_t>& fl = h->fl_cache;
    st.resize(top);
    fl.resize(top);
    if (top > 0) {
        PCHK(h, hipMemcpy(st.data(), h->d_st, top * sizeof(DevParticle), hipMemcpyDeviceToHost));
        PCHK(h, hipMemcpy(fl.data(), h->d_flags, top * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    h->cache_valid = true;
    for (auto& kv : h->members) {
        Member& m = *kv.second;
        m.steps_done = st[m.lane].step;
        const int32_t before = m.state;
        if (fl[m.lane])
            m.state = LBIB_POOL_FAILED;
        else if (m.steps_done >= m.target)
            m.state = LBIB_POOL_FINISHED;
        if (m.state != before) h->dirty = true;
    }
    return LBIB_OK;
}

std::string flag_text(int32_t fl)
{
    std::string m;
    if (fl & FLAG_NONFINITE) m += " non-finite force/torque/velocity;";
    if (fl & FLAG_CONTACT) m += " particle touches the receptor wall (gap <= 0);";
    if (fl & FLAG_MLS) m += " singular MLS moment matrix;";
    if (fl & FLAG_TILE) m += " spread footprint exceeds the tile;";
    if (fl & FLAG_SYNC) m += " grid barrier timed out;";
    return m;
}

}  // namespace

extern "C" {

lbib_status lbib_pool_create(int32_t precision, int64_t hbm_budget_bytes, int32_t max_members, void* hip_stream,
                             lbib_pool_handle* out)
{
    if (!out) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_create: NULL output");
    if (precision < LBIB_FP64 || precision > LBIB_BF16_NEQ)
        return fail(nullptr, LBIB_E_UNSUPPORTED,
                    "lbib_pool_create: precision must be LBIB_FP64, LBIB_FP32, LBIB_FP16, LBIB_BF16, LBIB_FP16_NEQ or "
                    "LBIB_BF16_NEQ");
    if (hbm_budget_bytes <= 0) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_create: budget must be positive");
    if (max_members < 1 || max_members > 65536)
        return fail(nullptr, LBIB_E_INVALID, "lbib_pool_create: max_members must be in [1, 65536]");
    lbib_pool* h = nullptr;
    try {
        h = new lbib_pool();
        h->precision = precision;
        h->elem = precision == LBIB_FP64 ? 8 : precision == LBIB_FP32 ? 4 : 2;
        h->budget = hbm_budget_bytes;
        h->max_members = max_members;
        for (int32_t l = max_members - 1; l >= 0; --l) h->free_lanes.push_back(l);
    } catch (const std::bad_alloc&) {
        delete h;
        return fail(nullptr, LBIB_E_NOMEM, "lbib_pool_create: host allocation failed");
    }
    hipError_t e;
    if ((e = dalloc(&h->d_st, (size_t)max_members)) != hipSuccess ||
        (e = dalloc(&h->d_flags, (size_t)max_members)) != hipSuccess) {
        dfree(h->d_st);
        delete h;
        return hip_fail(nullptr, e, "lbib_pool_create: device allocation");
    }
    if ((e = hipMemset(h->d_flags, 0, (size_t)max_members * sizeof(int32_t))) != hipSuccess ||
        (e = hipMemset(h->d_st, 0, (size_t)max_members * sizeof(DevParticle))) != hipSuccess ||
        (e = h->arena.init((size_t)hbm_budget_bytes)) != hipSuccess) {
        dfree(h->d_st);
        dfree(h->d_flags);
        delete h;
        return hip_fail(nullptr, e, "lbib_pool_create: device allocation of the budget");
    }
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess) {
            dfree(h->d_st);
            dfree(h->d_flags);
            delete h;
            return hip_fail(nullptr, e, "lbib_pool_create: hipStreamCreate");
        }
        h->own_stream = true;
    }
    *out = h;
    return LBIB_OK;
}

lbib_status lbib_pool_footprint(const lbib_lattice_desc* lat, const lbib_particle_desc* pd, int64_t* bytes)
{
    if (!lat || !pd || !bytes) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_footprint: NULL argument");
    std::string msg;
    lbib_status s = check_lattice(*lat, msg);
    if (s != LBIB_OK) return fail(nullptr, s, "lbib_pool_footprint: " + msg);
    try {
        Particle p;
        s = prepare_particle(*lat, *pd, p, msg);
        if (s != LBIB_OK) return fail(nullptr, s, "lbib_pool_footprint: " + msg);
        *bytes = footprint_bytes(*lat, &p);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, LBIB_E_NOMEM, "lbib_pool_footprint: host allocation failed");
    }
    return LBIB_OK;
}

lbib_status lbib_pool_add(lbib_pool_handle h, const lbib_lattice_desc* lat, const lbib_particle_desc* pd,
                          const lbib_ligand_desc* lig, int64_t n_steps, int32_t* slot)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_add: NULL handle");
    if (!lat || !pd || !lig || !slot) return fail(h, LBIB_E_INVALID, "lbib_pool_add: NULL argument");
    if (n_steps < 0) return fail(h, LBIB_E_INVALID, "lbib_pool_add: negative step count");
    std::string msg;
    lbib_status s = check_lattice(*lat, msg);
    if (s != LBIB_OK) return fail(h, s, "lbib_pool_add: " + msg);
    if (lat->precision != h->precision)
        return fail(h, LBIB_E_INVALID, "lbib_pool_add: lattice precision differs from the pool's");
    if ((s = check_ligands(*lig, msg)) != LBIB_OK) return fail(h, s, "lbib_pool_add: " + msg);
    std::unique_ptr<Member> m;
    try {
        m.reset(new Member());
        if ((s = prepare_particle(*lat, *pd, m->p, msg)) != LBIB_OK) return fail(h, s, "lbib_pool_add: " + msg);
        set_ligands(m->p, *lig);
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_pool_add: host allocation failed");
    }
    m->lat = *lat;
    m->g = lattice_geom(*lat);
    m->g.pull = true;  // the pool sweep runs the pull update
    m->target = n_steps;
    m->bytes = footprint_bytes(*lat, &m->p);
    if (h->free_lanes.empty()) return fail(h, LBIB_E_FULL, "lbib_pool_add: max_members members already in the pool");
    if (h->in_use + m->bytes > h->budget)
        return fail(h, LBIB_E_FULL,
                    "lbib_pool_add: needs " + std::to_string(m->bytes) + " bytes, " +
                        std::to_string(h->budget - h->in_use) + " left in the budget");
    m->block = h->arena.alloc((size_t)m->bytes);
    if (!m->block) return fail(h, LBIB_E_FULL, "lbib_pool_add: no contiguous free block of the budget is large enough");
    const size_t pop = align_up(m->g.buf_bytes);
    m->fA = m->block;
    m->fB = m->block + pop;
    carve_particle(m->p, m->block + 2 * pop);
    m->lane = h->free_lanes.back();
    m->p.d_st = h->d_st + m->lane;  // the pool-wide lane replaces the block's own state slot
    // everything below is stream-ordered: the member's first step sees it complete
    hipError_t e;
    auto bail = [&](hipError_t err, const char* what) {
        (void)hipStreamSynchronize(h->stream);
        free_member(h, *m);
        return hip_fail(h, err, what);
    };
    if ((e = hipMemsetAsync(m->fB, 0, pop, h->stream)) != hipSuccess) return bail(e, "lbib_pool_add: hipMemset");
    if ((e = hipMemsetAsync(h->d_flags + m->lane, 0, sizeof(int32_t), h->stream)) != hipSuccess)
        return bail(e, "lbib_pool_add: hipMemset");
    if ((e = init_populations(m->fA, m->g, h->stream)) != hipSuccess) return bail(e, "lbib_pool_add: init kernel");
    if ((e = upload_particle(m->p, h->stream)) != hipSuccess) return bail(e, "lbib_pool_add: upload");
    h->cache_valid = false;
    h->free_lanes.pop_back();
    m->slot = h->next_slot++;
    m->state = n_steps > 0 ? LBIB_POOL_RUNNING : LBIB_POOL_FINISHED;
    h->in_use += m->bytes;
    *slot = m->slot;
    h->members[m->slot] = std::move(m);
    h->dirty = true;
    return LBIB_OK;
}

lbib_status lbib_pool_step(lbib_pool_handle h, int64_t n)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_step: NULL handle");
    if (n < 0) return fail(h, LBIB_E_INVALID, "lbib_pool_step: negative step count");
    switch (h->precision) {
        case LBIB_FP64: return enqueue<double>(h, n);
        case LBIB_FP32: return enqueue<float>(h, n);
        case LBIB_FP16: return enqueue<half_t>(h, n);
        case LBIB_BF16: return enqueue<bf16_t>(h, n);
        case LBIB_FP16_NEQ: return enqueue<half_neq_t>(h, n);
        default: return enqueue<bf16_neq_t>(h, n);
    }
}

lbib_status lbib_pool_poll(lbib_pool_handle h, int32_t* slots, int32_t capacity, int32_t* count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_poll: NULL handle");
    if (!count || capacity < 0 || (capacity > 0 && !slots))
        return fail(h, LBIB_E_INVALID, "lbib_pool_poll: NULL output or negative capacity");
    lbib_status s = refresh(h);
    if (s != LBIB_OK) return s;
    int32_t n = 0;
    for (auto& kv : h->members) {
        Member& m = *kv.second;
        if (m.state == LBIB_POOL_RUNNING || m.reported || n >= capacity) continue;
        slots[n++] = m.slot;
        m.reported = true;
    }
    *count = n;
    return LBIB_OK;
}

lbib_status lbib_pool_status(lbib_pool_handle h, int32_t slot, int64_t* steps_done, int32_t* state)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_status: NULL handle");
    if (!steps_done || !state) return fail(h, LBIB_E_INVALID, "lbib_pool_status: NULL output");
    if (!get_member(h, slot)) return fail(h, LBIB_E_INVALID, "lbib_pool_status: unknown slot");
    lbib_status s = refresh(h);
    if (s != LBIB_OK) return s;
    Member* m = get_member(h, slot);
    *steps_done = m->steps_done;
    *state = m->state;
    if (m->state == LBIB_POOL_FAILED)
        h->err = "lbib_pool_status: slot " + std::to_string(slot) + " failed:" + flag_text(h->fl_cache[m->lane]);
    return LBIB_OK;
}

lbib_status lbib_pool_read_particle(lbib_pool_handle h, int32_t slot, lbib_particle_state* out)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_read_particle: NULL handle");
    Member* m = get_member(h, slot);
    if (!m || !out) return fail(h, LBIB_E_INVALID, "lbib_pool_read_particle: unknown slot or NULL output");
    lbib_status s = refresh(h);
    if (s != LBIB_OK) return s;
    *out = h->st_cache[m->lane].last;
    return LBIB_OK;
}

lbib_status lbib_pool_read_bonds(lbib_pool_handle h, int32_t slot, uint8_t* bonded, uint8_t* ligand, int32_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_read_bonds: NULL handle");
    Member* m = get_member(h, slot);
    if (!m) return fail(h, LBIB_E_INVALID, "lbib_pool_read_bonds: unknown slot");
    if (capacity < m->p.nl)
        return fail(h, LBIB_E_INVALID, "lbib_pool_read_bonds: capacity must be >= " + std::to_string(m->p.nl));
    PCHK(h, hipStreamSynchronize(h->stream));
    if (bonded) PCHK(h, hipMemcpy(bonded, m->p.d_bond, m->p.nl, hipMemcpyDeviceToHost));
    if (ligand) std::memcpy(ligand, m->p.ligand.data(), m->p.nl);
    return LBIB_OK;
}

lbib_status lbib_pool_read_field(lbib_pool_handle h, int32_t slot, int32_t which, double* out, int64_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_read_field: NULL handle");
    Member* m = get_member(h, slot);
    if (!m || !out) return fail(h, LBIB_E_INVALID, "lbib_pool_read_field: unknown slot or NULL output");
    if (which < 0 || which > 3) return fail(h, LBIB_E_INVALID, "lbib_pool_read_field: which must be 0..3");
    const int64_t need = (which == 3 ? 9 : 1) * (int64_t)m->g.nx * m->g.ny;
    if (capacity < need)
        return fail(h, LBIB_E_INVALID, "lbib_pool_read_field: capacity must be >= " + std::to_string(need));
    try {
        PCHK(h, hipStreamSynchronize(h->stream));
        DevParticle st;
        PCHK(h, hipMemcpy(&st, m->p.d_st, sizeof(st), hipMemcpyDeviceToHost));
        std::vector<double> f;
        PCHK(h, download_populations((st.step & 1) ? m->fB : m->fA, m->g, f));
        field_from_populations(f, m->g, which, out);
    } catch (const std::bad_alloc&) {
        return fail(h, LBIB_E_NOMEM, "lbib_pool_read_field: host allocation failed");
    }
    return LBIB_OK;
}

lbib_status lbib_pool_trace_enable(lbib_pool_handle h, int32_t slot, int64_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_trace_enable: NULL handle");
    Member* m = get_member(h, slot);
    if (!m) return fail(h, LBIB_E_INVALID, "lbib_pool_trace_enable: unknown slot");
    if (capacity < 0 || capacity > ((int64_t)1 << 28))
        return fail(h, LBIB_E_INVALID, "lbib_pool_trace_enable: capacity must be in [0, 2^28]");
    PCHK(h, hipStreamSynchronize(h->stream));
    DevParticle st;
    PCHK(h, hipMemcpy(&st, m->p.d_st, sizeof(st), hipMemcpyDeviceToHost));
    dfree(m->p.d_trace);
    m->p.trace_cap = 0;
    if (capacity > 0) {
        hipError_t e = dalloc(&m->p.d_trace, (size_t)capacity);
        if (e != hipSuccess) return hip_fail(h, e, "lbib_pool_trace_enable: allocation");
        m->p.trace_cap = capacity;
    }
    m->p.trace_start = st.step;
    h->dirty = true;
    return LBIB_OK;
}

lbib_status lbib_pool_read_trace(lbib_pool_handle h, int32_t slot, lbib_particle_state* out, int64_t capacity,
                                 int64_t* count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_read_trace: NULL handle");
    Member* m = get_member(h, slot);
    if (!m || !out || !count) return fail(h, LBIB_E_INVALID, "lbib_pool_read_trace: unknown slot or NULL output");
    PCHK(h, hipStreamSynchronize(h->stream));
    DevParticle st;
    PCHK(h, hipMemcpy(&st, m->p.d_st, sizeof(st), hipMemcpyDeviceToHost));
    const int64_t have = std::min(m->p.trace_cap, std::max<int64_t>(0, st.step - m->p.trace_start));
    const int64_t n = std::min(have, capacity);
    if (n > 0) PCHK(h, hipMemcpy(out, m->p.d_trace, (size_t)n * sizeof(lbib_particle_state), hipMemcpyDeviceToHost));
    *count = n;
    return LBIB_OK;
}

lbib_status lbib_pool_remove(lbib_pool_handle h, int32_t slot)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_remove: NULL handle");
    auto it = h->members.find(slot);
    if (it == h->members.end()) return fail(h, LBIB_E_INVALID, "lbib_pool_remove: unknown slot");
    PCHK(h, hipStreamSynchronize(h->stream));  // no enqueued step may still use its buffers
    Member& m = *it->second;
    free_member(h, m);
    h->free_lanes.push_back(m.lane);
    h->in_use -= m.bytes;
    h->members.erase(it);
    h->dirty = true;
    return LBIB_OK;
}

lbib_status lbib_pool_usage(lbib_pool_handle h, int32_t* members, int32_t* running, int64_t* bytes_in_use)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_usage: NULL handle");
    if (!members || !running || !bytes_in_use) return fail(h, LBIB_E_INVALID, "lbib_pool_usage: NULL output");
    int32_t r = 0;
    for (auto& kv : h->members) r += kv.second->state == LBIB_POOL_RUNNING;
    *members = (int32_t)h->members.size();
    *running = r;
    *bytes_in_use = h->in_use;
    return LBIB_OK;
}

lbib_status lbib_pool_kernel_timing(lbib_pool_handle h, int32_t enable)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_kernel_timing: NULL handle");
    PCHK(h, hipStreamSynchronize(h->stream));
    if (enable) {
        for (int k = 0; k < 2; ++k) {
            while (h->ev[k].size() < (size_t)2 * kPoolTimingPool) {
                hipEvent_t e;
                PCHK(h, hipEventCreate(&e));
                h->ev[k].push_back(e);
            }
            h->ev_used[k] = 0;
            h->launches[k] = 0;
        }
    }
    h->timing = enable != 0;
    return LBIB_OK;
}

lbib_status lbib_pool_kernel_time(lbib_pool_handle h, int32_t kernel, double* total_ms, int64_t* launches)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_kernel_time: NULL handle");
    if (kernel < 0 || kernel > 1 || !total_ms || !launches)
        return fail(h, LBIB_E_INVALID, "lbib_pool_kernel_time: kernel must be 0 or 1 and outputs non-NULL");
    PCHK(h, hipStreamSynchronize(h->stream));
    double acc = 0.0;
    for (size_t k = 0; k + 1 < h->ev_used[kernel]; k += 2) {
        float ms = 0.0f;
        PCHK(h, hipEventElapsedTime(&ms, h->ev[kernel][k], h->ev[kernel][k + 1]));
        acc += ms;
    }
    *total_ms = acc;
    *launches = h->launches[kernel];
    return LBIB_OK;
}

lbib_status lbib_pool_set_config(lbib_pool_handle h, int32_t tile_x, int32_t tiles_per_block, int32_t graph_steps)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_set_config: NULL handle");
    if (!valid_config(tile_x, tiles_per_block) || graph_steps < 0 || graph_steps > 4096)
        return fail(h, LBIB_E_INVALID,
                    "lbib_pool_set_config: tile_x in {64, 128, 256}, tiles_per_block in {1, 2, 4, 8}, "
                    "graph_steps in [0, 4096]");
    PCHK(h, hipStreamSynchronize(h->stream));
    h->cfg = PoolSweepConfig{tile_x, tiles_per_block};
    h->graph_steps = graph_steps;
    h->dirty = true;
    return LBIB_OK;
}

lbib_status lbib_pool_get_config(lbib_pool_handle h, int32_t* tile_x, int32_t* tiles_per_block, int32_t* graph_steps)
{
    if (!h || !tile_x || !tiles_per_block || !graph_steps)
        return fail(h, LBIB_E_INVALID, "lbib_pool_get_config: NULL argument");
    *tile_x = h->cfg.bx;
    *tiles_per_block = h->cfg.tpb;
    *graph_steps = h->graph_steps;
    return LBIB_OK;
}

lbib_status lbib_pool_autotune(lbib_pool_handle h, int32_t steps_per_trial, double* best_step_us)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_pool_autotune: NULL handle");
    if (steps_per_trial < 1 || steps_per_trial > 100000)
        return fail(h, LBIB_E_INVALID, "lbib_pool_autotune: steps_per_trial must be in [1, 100000]");
    // sweep duration of one configuration: HIP events around each sweep launch (they do not
    // change a kernel's own duration), after 2 untimed steps for the table rebuild
    auto sweep_trial = [&](PoolSweepConfig c, double& us) -> lbib_status {
        PCHK(h, hipStreamSynchronize(h->stream));
        h->cfg = c;
        h->graph_steps = 0;
        h->dirty = true;
        h->timing = false;
        lbib_status s = lbib_pool_step(h, 2);
        if (s != LBIB_OK) return s;
        if ((s = lbib_pool_kernel_timing(h, 1)) != LBIB_OK) return s;
        if ((s = lbib_pool_step(h, steps_per_trial)) != LBIB_OK) return s;
        double ms = 0;
        int64_t n = 0;
        if ((s = lbib_pool_kernel_time(h, 0, &ms, &n)) != LBIB_OK) return s;
        h->timing = false;
        us = n > 0 ? ms * 1e3 / n : 1e300;
        return LBIB_OK;
    };
    // whole steps, wall clock, with or without graph replay
    auto step_trial = [&](int32_t gsteps, double& us) -> lbib_status {
        PCHK(h, hipStreamSynchronize(h->stream));
        h->graph_steps = gsteps;
        h->dirty = true;
        h->timing = false;
        lbib_status s = lbib_pool_step(h, std::max<int32_t>(2, gsteps));  // rebuild and capture off the clock
        if (s != LBIB_OK) return s;
        PCHK(h, hipStreamSynchronize(h->stream));
        const int64_t n = gsteps > 0 ? (steps_per_trial + gsteps - 1) / gsteps * gsteps : steps_per_trial;
        const auto t0 = std::chrono::steady_clock::now();
        if ((s = lbib_pool_step(h, n)) != LBIB_OK) return s;
        PCHK(h, hipStreamSynchronize(h->stream));
        us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() / n;
        return LBIB_OK;
    };
    static const PoolSweepConfig cand[] = {{64, 1},  {64, 2},  {64, 4},  {64, 8},  {128, 1}, {128, 2},
                                           {128, 4}, {128, 8}, {256, 1}, {256, 2}, {256, 4}, {256, 8}};
    constexpr int kCand = sizeof(cand) / sizeof(cand[0]);
    double best_sweep[kCand];
    for (int c = 0; c < kCand; ++c) best_sweep[c] = 1e300;
    for (int round = 0; round < 2; ++round)  // two rounds, best of each: drifts in clock hit every shape
        for (int c = 0; c < kCand; ++c) {
            double us = 0;
            lbib_status s = sweep_trial(cand[c], us);
            if (s != LBIB_OK) return s;
            best_sweep[c] = std::min(best_sweep[c], us);
        }
    int bi = 0;
    for (int c = 1; c < kCand; ++c)
        if (best_sweep[c] < best_sweep[bi]) bi = c;
    h->cfg = cand[bi];
    const int32_t g = std::min<int32_t>(steps_per_trial, 64);
    double direct = 1e300, graphed = 1e300;
    for (int round = 0; round < 2; ++round) {
        double us = 0;
        lbib_status s = step_trial(0, us);
        if (s != LBIB_OK) return s;
        direct = std::min(direct, us);
        if ((s = step_trial(g, us)) != LBIB_OK) return s;
        graphed = std::min(graphed, us);
    }
    h->graph_steps = graphed < direct ? g : 0;
    h->dirty = true;
    h->timing = false;
    if (best_step_us) *best_step_us = std::min(direct, graphed);
    return LBIB_OK;
}

const char* lbib_pool_last_error(lbib_pool_handle h) { return h ? h->err.c_str() : g_pool_null_err.c_str(); }

void lbib_pool_destroy(lbib_pool_handle h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->members) free_member(h, *kv.second);
    h->members.clear();
    h->arena.release();
    dfree(h->d_st);
    dfree(h->d_flags);
    if (h->d_args) (void)hipFree(h->d_args);
    if (h->d_sims) (void)hipFree(h->d_sims);
    dfree(h->d_active);
    dfree(h->d_table);
    dfree(h->d_ctl);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    for (int k = 0; k < 2; ++k)
        for (auto e : h->ev[k]) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // extern "C"
