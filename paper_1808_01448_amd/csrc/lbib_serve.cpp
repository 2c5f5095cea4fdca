// lbib_serve.cpp -- continuous-batching request loop over a pool.  Each request is one
// adhesion solve (lattice, particle, ligands, step count); requests queue on the host in
// arrival order and are admitted into the pool as soon as a slot and enough of the memory
// budget are free, while the requests already admitted keep stepping on the GPU.  Finished
// solves are collected after every chunk of steps and leave the pool at once, freeing their
// memory for the next admissions.  Implements the server part of include/lbib.h.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lbib.h"

namespace {

struct Request {
    int64_t id = 0;
    lbib_lattice_desc lat{};
    lbib_particle_desc part{};
    lbib_ligand_desc lig{};
    int64_t steps = 0;
    int64_t bytes = 0;
    int32_t bypassed = 0;  // admissions of later requests while this one waited at the head
    lbib_request_result res{};
    // copied out of the pool when the request completes (before it leaves): the bond and
    // ligand flags after its last step and, when tracing was on at admission, its records
    std::vector<uint8_t> bonded, ligand;
    std::vector<lbib_particle_state> trace;
    int64_t trace_cap = 0;
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct lbib_server {
    lbib_pool_handle pool = nullptr;
    int32_t chunk = 0;
    int32_t max_bypass = 0;
    int64_t budget = 0;
    std::chrono::steady_clock::time_point t0;
    int64_t next_id = 0;
    std::deque<Request*> queue;              // waiting, in arrival order
    std::map<int32_t, Request*> running;     // pool slot -> request
    std::map<int64_t, Request*> all;         // every request not yet released
    std::vector<int64_t> completed;          // finished or failed, not yet taken
    std::string err;
    int64_t chunks = 0;
    int64_t trace_cap = 0;  // records kept per request admitted from now on (0: none)
};

namespace {

thread_local std::string g_srv_null_err;

lbib_status fail(lbib_server* h, lbib_status s, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_srv_null_err = msg;
    return s;
}

lbib_status pool_fail(lbib_server* h, lbib_status s, const char* what)
{
    return fail(h, s, std::string(what) + ": " + lbib_pool_last_error(h->pool));
}

// Admit waiting requests, first fit in arrival order: a request that does not fit the free
// memory is passed over by later ones that do, but at most max_bypass times; then nothing
// behind it is admitted until it is.
lbib_status admit(lbib_server* h)
{
    int32_t members = 0, running = 0;
    int64_t used = 0;
    lbib_status s = lbib_pool_usage(h->pool, &members, &running, &used);
    if (s != LBIB_OK) return pool_fail(h, s, "lbib_server: usage");
    for (auto it = h->queue.begin(); it != h->queue.end();) {
        Request* r = *it;
        const bool head = it == h->queue.begin();
        if (used + r->bytes > h->budget) {
            if (head && r->bypassed >= h->max_bypass) break;
            ++it;
            continue;
        }
        int32_t slot = -1;
        s = lbib_pool_add(h->pool, &r->lat, &r->part, &r->lig, r->steps, &slot);
        if (s == LBIB_E_FULL) break;  // out of slots: nothing else can join now
        if (s != LBIB_OK) {
            // a request the pool refuses (its descriptors were checked at submission, so this
            // is a device failure) is completed as failed
            r->res.state = LBIB_REQ_FAILED;
            r->res.t_done = now_s(h->t0);
            h->completed.push_back(r->id);
            it = h->queue.erase(it);
            continue;
        }
        if (h->trace_cap > 0) {
            r->trace_cap = std::min(h->trace_cap, r->steps);
            if ((s = lbib_pool_trace_enable(h->pool, slot, r->trace_cap)) != LBIB_OK)
                return pool_fail(h, s, "lbib_server: trace");
        }
        r->res.state = LBIB_REQ_RUNNING;
        r->res.t_admit = now_s(h->t0);
        r->res.slot = slot;
        used += r->bytes;
        h->running[slot] = r;
        if (!head) h->queue.front()->bypassed += 1;
        it = h->queue.erase(it);
    }
    return LBIB_OK;
}

lbib_status collect(lbib_server* h)
{
    std::vector<int32_t> done(h->running.size() + 1);
    int32_t n = 0;
    lbib_status s = lbib_pool_poll(h->pool, done.data(), (int32_t)done.size(), &n);
    if (s != LBIB_OK) return pool_fail(h, s, "lbib_server: poll");
    const double t = now_s(h->t0);
    for (int32_t k = 0; k < n; ++k) {
        auto it = h->running.find(done[k]);
        if (it == h->running.end()) continue;
        Request* r = it->second;
        int64_t steps = 0;
        int32_t state = 0;
        if ((s = lbib_pool_status(h->pool, done[k], &steps, &state)) != LBIB_OK)
            return pool_fail(h, s, "lbib_server: status");
        if ((s = lbib_pool_read_particle(h->pool, done[k], &r->res.final_state)) != LBIB_OK)
            return pool_fail(h, s, "lbib_server: read");
        const int32_t nl = r->part.n_markers;
        r->bonded.assign((size_t)nl, 0);
        r->ligand.assign((size_t)nl, 0);
        if ((s = lbib_pool_read_bonds(h->pool, done[k], r->bonded.data(), r->ligand.data(), nl)) != LBIB_OK)
            return pool_fail(h, s, "lbib_server: bonds");
        if (r->trace_cap > 0) {
            int64_t cnt = 0;
            r->trace.resize((size_t)r->trace_cap);
            if ((s = lbib_pool_read_trace(h->pool, done[k], r->trace.data(), r->trace_cap, &cnt)) != LBIB_OK)
                return pool_fail(h, s, "lbib_server: trace");
            r->trace.resize((size_t)cnt);
        }
        r->res.steps_done = steps;
        r->res.state = state == LBIB_POOL_FINISHED ? LBIB_REQ_DONE : LBIB_REQ_FAILED;
        r->res.t_done = t;
        r->res.slot = -1;
        if ((s = lbib_pool_remove(h->pool, done[k])) != LBIB_OK) return pool_fail(h, s, "lbib_server: remove");
        h->running.erase(it);
        h->completed.push_back(r->id);
    }
    return LBIB_OK;
}

// A completed request, or nullptr with the error set.
Request* completed_request(lbib_server* h, int64_t id, const char* what)
{
    auto it = h->all.find(id);
    if (it == h->all.end()) {
        fail(h, LBIB_E_INVALID, std::string(what) + ": unknown or released request");
        return nullptr;
    }
    const int32_t st = it->second->res.state;
    if (st != LBIB_REQ_DONE && st != LBIB_REQ_FAILED) {
        fail(h, LBIB_E_STATE, std::string(what) + ": the request has not completed");
        return nullptr;
    }
    return it->second;
}

}  // namespace

extern "C" {

lbib_status lbib_server_create(int32_t precision, int64_t hbm_budget_bytes, int32_t max_members, int32_t chunk_steps,
                               int32_t max_bypass, void* hip_stream, lbib_server_handle* out)
{
    if (!out) return fail(nullptr, LBIB_E_INVALID, "lbib_server_create: NULL output");
    if (chunk_steps < 1 || chunk_steps > 1000000)
        return fail(nullptr, LBIB_E_INVALID, "lbib_server_create: chunk_steps must be in [1, 10^6]");
    if (max_bypass < 0) return fail(nullptr, LBIB_E_INVALID, "lbib_server_create: max_bypass must be >= 0");
    lbib_server* h = nullptr;
    try {
        h = new lbib_server();
    } catch (const std::bad_alloc&) {
        return fail(nullptr, LBIB_E_NOMEM, "lbib_server_create: host allocation failed");
    }
    lbib_status s = lbib_pool_create(precision, hbm_budget_bytes, max_members, hip_stream, &h->pool);
    if (s != LBIB_OK) {
        std::string m = std::string("lbib_server_create: ") + lbib_pool_last_error(nullptr);
        delete h;
        return fail(nullptr, s, m);
    }
    h->chunk = chunk_steps;
    h->max_bypass = max_bypass;
    h->budget = hbm_budget_bytes;
    h->t0 = std::chrono::steady_clock::now();
    *out = h;
    return LBIB_OK;
}

lbib_status lbib_server_submit(lbib_server_handle h, const lbib_lattice_desc* lat, const lbib_particle_desc* part,
                               const lbib_ligand_desc* lig, int64_t n_steps, double arrival_s, int64_t* id)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_submit: NULL handle");
    if (!lat || !part || !lig || !id) return fail(h, LBIB_E_INVALID, "lbib_server_submit: NULL argument");
    if (n_steps < 0) return fail(h, LBIB_E_INVALID, "lbib_server_submit: negative step count");
    int64_t bytes = 0;
    lbib_status s = lbib_pool_footprint(lat, part, &bytes);
    if (s != LBIB_OK) return fail(h, s, std::string("lbib_server_submit: ") + lbib_pool_last_error(nullptr));
    if (bytes > h->budget)
        return fail(h, LBIB_E_FULL, "lbib_server_submit: the request alone exceeds the memory budget");
    Request* r = nullptr;
    try {
        r = new Request();
        r->id = h->next_id;
        r->lat = *lat;
        r->part = *part;
        r->lig = *lig;
        r->steps = n_steps;
        r->bytes = bytes;
        r->res.id = r->id;
        r->res.state = LBIB_REQ_QUEUED;
        r->res.steps = n_steps;
        r->res.bytes = bytes;
        r->res.slot = -1;
        r->res.t_arrival = arrival_s >= 0 ? arrival_s : now_s(h->t0);
        r->res.t_submit = now_s(h->t0);
        r->res.final_state.step = -1;
        h->queue.push_back(r);
        h->all[r->id] = r;
    } catch (const std::bad_alloc&) {
        delete r;
        return fail(h, LBIB_E_NOMEM, "lbib_server_submit: host allocation failed");
    }
    h->next_id += 1;
    *id = r->id;
    return LBIB_OK;
}

lbib_status lbib_server_progress(lbib_server_handle h, int32_t* n_completed)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_progress: NULL handle");
    lbib_status s = admit(h);
    if (s != LBIB_OK) return s;
    if (!h->running.empty()) {
        if ((s = lbib_pool_step(h->pool, h->chunk)) != LBIB_OK) return pool_fail(h, s, "lbib_server: step");
        h->chunks += 1;
    }
    if ((s = collect(h)) != LBIB_OK) return s;
    if (n_completed) *n_completed = (int32_t)h->completed.size();
    return LBIB_OK;
}

lbib_status lbib_server_take_completed(lbib_server_handle h, int64_t* ids, int32_t capacity, int32_t* count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_take_completed: NULL handle");
    if (!count || capacity < 0 || (capacity > 0 && !ids))
        return fail(h, LBIB_E_INVALID, "lbib_server_take_completed: NULL output or negative capacity");
    const int32_t n = std::min<int32_t>(capacity, (int32_t)h->completed.size());
    std::copy(h->completed.begin(), h->completed.begin() + n, ids);
    h->completed.erase(h->completed.begin(), h->completed.begin() + n);
    *count = n;
    return LBIB_OK;
}

lbib_status lbib_server_result(lbib_server_handle h, int64_t id, lbib_request_result* out)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_result: NULL handle");
    if (!out) return fail(h, LBIB_E_INVALID, "lbib_server_result: NULL output");
    auto it = h->all.find(id);
    if (it == h->all.end()) return fail(h, LBIB_E_INVALID, "lbib_server_result: unknown or released request");
    *out = it->second->res;
    return LBIB_OK;
}

lbib_status lbib_server_set_trace(lbib_server_handle h, int64_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_set_trace: NULL handle");
    if (capacity < 0 || capacity > ((int64_t)1 << 28))
        return fail(h, LBIB_E_INVALID, "lbib_server_set_trace: capacity must be in [0, 2^28]");
    h->trace_cap = capacity;
    return LBIB_OK;
}

lbib_status lbib_server_read_trace(lbib_server_handle h, int64_t id, lbib_particle_state* out, int64_t capacity,
                                   int64_t* count)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_read_trace: NULL handle");
    if (!count || capacity < 0 || (capacity > 0 && !out))
        return fail(h, LBIB_E_INVALID, "lbib_server_read_trace: NULL output or negative capacity");
    Request* r = completed_request(h, id, "lbib_server_read_trace");
    if (!r) return h->all.count(id) ? LBIB_E_STATE : LBIB_E_INVALID;
    const int64_t n = std::min<int64_t>(capacity, (int64_t)r->trace.size());
    std::copy(r->trace.begin(), r->trace.begin() + n, out);
    *count = n;
    return LBIB_OK;
}

lbib_status lbib_server_read_bonds(lbib_server_handle h, int64_t id, uint8_t* bonded, uint8_t* ligand,
                                   int32_t capacity)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_read_bonds: NULL handle");
    Request* r = completed_request(h, id, "lbib_server_read_bonds");
    if (!r) return h->all.count(id) ? LBIB_E_STATE : LBIB_E_INVALID;
    const int32_t nl = (int32_t)r->bonded.size();
    if (capacity < nl)
        return fail(h, LBIB_E_INVALID, "lbib_server_read_bonds: capacity below n_markers = " + std::to_string(nl));
    if (bonded) std::copy(r->bonded.begin(), r->bonded.end(), bonded);
    if (ligand) std::copy(r->ligand.begin(), r->ligand.end(), ligand);
    return LBIB_OK;
}

lbib_status lbib_server_release(lbib_server_handle h, int64_t id)
{
    if (!h) return fail(nullptr, LBIB_E_INVALID, "lbib_server_release: NULL handle");
    auto it = h->all.find(id);
    if (it == h->all.end()) return fail(h, LBIB_E_INVALID, "lbib_server_release: unknown or released request");
    const int32_t st = it->second->res.state;
    if (st != LBIB_REQ_DONE && st != LBIB_REQ_FAILED)
        return fail(h, LBIB_E_STATE, "lbib_server_release: the request has not completed");
    delete it->second;
    h->all.erase(it);
    return LBIB_OK;
}

lbib_status lbib_server_stats(lbib_server_handle h, int32_t* queued, int32_t* running, int64_t* bytes_in_use,
                              int64_t* chunks)
{
    if (!h || !queued || !running || !bytes_in_use || !chunks)
        return fail(h, LBIB_E_INVALID, "lbib_server_stats: NULL argument");
    int32_t members = 0, run = 0;
    lbib_status s = lbib_pool_usage(h->pool, &members, &run, bytes_in_use);
    if (s != LBIB_OK) return pool_fail(h, s, "lbib_server_stats");
    *queued = (int32_t)h->queue.size();
    *running = (int32_t)h->running.size();
    *chunks = h->chunks;
    return LBIB_OK;
}

lbib_pool_handle lbib_server_pool(lbib_server_handle h) { return h ? h->pool : nullptr; }

double lbib_server_clock(lbib_server_handle h) { return h ? now_s(h->t0) : 0.0; }

const char* lbib_server_last_error(lbib_server_handle h) { return h ? h->err.c_str() : g_srv_null_err.c_str(); }

void lbib_server_destroy(lbib_server_handle h)
{
    if (!h) return;
    lbib_pool_destroy(h->pool);
    for (auto& kv : h->all) delete kv.second;
    delete h;
}

}  // extern "C"
