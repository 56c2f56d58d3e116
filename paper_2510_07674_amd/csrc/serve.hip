// Continuous-batching solve server (host side): requests are admitted in arrival order
// as slots and arena memory free up; an admitted request runs its prefix (stage 1, lift,
// seeding) and its first chunk of stage-2 iterations on the admission stream while the
// running solves advance, and from the next step on it advances a chunk per step inside
// one batched launch per (thread count, sphere chunk) class.  Classes run on their own streams so that they
// overlap on the device, and each class's chunk is sized from its measured time per
// iteration so that a step takes about as long for every class: a small solve then
// advances many iterations while a large one advances a few.  Finished solves are retired
// with a completion record.  Device state of a solve (workspace and Adam moments) lives in
// the server's arena from admission to completion; only a 48-byte summary is copied back.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <utility>
#include <vector>

#include "spasm_internal.h"

using namespace spasm;

namespace {
struct Request {
    spasm_problem prob;
    spasm_solve_config cfg;
    uint64_t req_id;
    float *best_q, *best_pose;
};

struct Slot {
    bool used = false;
    bool ready = false;  // prefix done: takes part in the class launches
    bool fresh = false;  // admitted in this step: its first chunk follows its prefix on the admission stream
    Request r{};
    size_t off = 0, bytes = 0, opt_off = 0;
    SolveLayout L{};
    int k_done = 0, k_next = 0, steps = 0;
    bool finishing = false;
};

constexpr int N_CLASS_STREAMS = 4;
constexpr int MAX_CLASS_LAUNCHES = 64;  // timed class launches per step
constexpr double MIN_STEP_MS = 2.0;     // a step advances every class by at least this much work

using ClassKey = std::pair<int, int>;  // (threads, sphere chunk)

size_t opt_bytes(spasm_problem prob, const spasm_solve_config &c) { return stage2_opt_bytes(prob->kp, c); }

size_t request_footprint(spasm_problem prob, const spasm_solve_config &c)
{
    return align256(solve_layout(prob->kp, c).total) + align256(opt_bytes(prob, c));
}
}  // namespace

struct spasm_server_s {
    int device = 0;
    hipStream_t st = nullptr;                       // admission (prefix) work
    hipStream_t cs[N_CLASS_STREAMS] = {};           // class launches and finishing work
    hipEvent_t ev[2 * MAX_CLASS_LAUNCHES] = {};     // start / end of each class launch
    std::map<ClassKey, double> ms_per_iter;         // measured, smoothed
    size_t budget = 0;
    char *arena = nullptr;
    int iters = 25;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted by offset
    std::vector<Slot> slots;
    std::deque<Request> pending;
    std::deque<spasm_completion> done;
    ServeSolve *h_desc = nullptr;  // pinned, one per slot
    ServeSolve *d_desc = nullptr;
    int32_t *h_info = nullptr;     // pinned, 8 per slot
    float *h_finfo = nullptr;      // pinned, 4 per slot

    bool alloc(size_t n, size_t *off)
    {
        for (size_t i = 0; i < free_list.size(); ++i) {
            if (free_list[i].second >= n) {
                *off = free_list[i].first;
                free_list[i].first += n;
                free_list[i].second -= n;
                if (free_list[i].second == 0) free_list.erase(free_list.begin() + (long)i);
                return true;
            }
        }
        return false;
    }

    void release(size_t off, size_t n)
    {
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
        size_t i = (size_t)(free_list.insert(it, {off, n}) - free_list.begin());
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + (long)i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + (long)i);
        }
    }

    void cleanup()
    {
        if (st) (void)hipStreamSynchronize(st);
        for (auto &c : cs)
            if (c) {
                (void)hipStreamSynchronize(c);
                (void)hipStreamDestroy(c);
                c = nullptr;
            }
        for (auto &e : ev)
            if (e) {
                (void)hipEventDestroy(e);
                e = nullptr;
            }
        if (arena) (void)hipFree(arena);
        if (d_desc) (void)hipFree(d_desc);
        if (h_desc) (void)hipHostFree(h_desc);
        if (h_info) (void)hipHostFree(h_info);
        if (h_finfo) (void)hipHostFree(h_finfo);
        if (st) (void)hipStreamDestroy(st);
        arena = nullptr;
        d_desc = nullptr;
        h_desc = nullptr;
        h_info = nullptr;
        h_finfo = nullptr;
        st = nullptr;
    }
};

extern "C" size_t spasm_server_footprint(spasm_problem prob, const spasm_solve_config *cfg)
{
    if (check_cfg(prob, cfg)) return 0;
    return request_footprint(prob, *cfg);
}

extern "C" int spasm_server_create(size_t hbm_budget, int32_t max_slots, int32_t iters_per_step, spasm_server *out)
{
    if (!out) return fail(SPASM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096) return fail(SPASM_EINVAL, "max_slots=%d outside 1..4096", max_slots);
    if (iters_per_step < 1) return fail(SPASM_EINVAL, "iters_per_step must be >= 1");
    if (hbm_budget < 4096) return fail(SPASM_EINVAL, "hbm_budget too small");
    int rc = ensure_attrs();
    if (rc) return rc;
    auto *s = new spasm_server_s();
    s->budget = hbm_budget & ~(size_t)255;
    s->iters = iters_per_step;
    s->slots.resize((size_t)max_slots);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    for (int i = 0; i < N_CLASS_STREAMS && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&s->cs[i], hipStreamNonBlocking);
    for (int i = 0; i < 2 * MAX_CLASS_LAUNCHES && e == hipSuccess; ++i) e = hipEventCreate(&s->ev[i]);
    if (e != hipSuccess) {
        s->cleanup();
        delete s;
        return fail(SPASM_EHIP, "server stream: %s", hipGetErrorString(e));
    }
    if (hipMalloc(&s->arena, s->budget) != hipSuccess || hipMalloc(&s->d_desc, sizeof(ServeSolve) * max_slots) != hipSuccess ||
        hipHostMalloc(&s->h_desc, sizeof(ServeSolve) * max_slots) != hipSuccess ||
        hipHostMalloc(&s->h_info, sizeof(int32_t) * 8 * max_slots) != hipSuccess ||
        hipHostMalloc(&s->h_finfo, sizeof(float) * 4 * max_slots) != hipSuccess) {
        s->cleanup();
        delete s;
        return fail(SPASM_ENOMEM, "server allocation of %zu bytes failed", hbm_budget);
    }
    s->free_list.push_back({0, s->budget});
    *out = s;
    return SPASM_OK;
}

extern "C" int spasm_server_submit(spasm_server srv, spasm_problem prob, const spasm_solve_config *cfg, uint64_t req_id,
                                   float *d_best_q, float *d_best_pose)
{
    if (!srv) return fail(SPASM_EINVAL, "server is NULL");
    int rc = check_cfg(prob, cfg);
    if (rc) return rc;
    if (prob->kp.mode == SPASM_MODE_P2P)
        return fail(SPASM_EUNSUPPORTED, "the server takes manipulation solves; use spasm_solve for point to point");
    if (prob->kp.al_every > 0)
        return fail(SPASM_EUNSUPPORTED, "the server runs the plain penalty method (al_every = 0)");
    if (!d_best_q || !d_best_pose) return fail(SPASM_EINVAL, "NULL output buffer");
    if (prob->device != srv->device) return fail(SPASM_EINVAL, "problem lives on device %d, server on %d", prob->device, srv->device);
    const size_t need = request_footprint(prob, *cfg);
    if (need > srv->budget) return fail(SPASM_EBUSY, "request needs %zu bytes, the server has %zu", need, srv->budget);
    srv->pending.push_back(Request{prob, *cfg, req_id, d_best_q, d_best_pose});
    return SPASM_OK;
}

extern "C" int spasm_server_step(spasm_server srv, int32_t *n_active, int32_t *n_pending)
{
    if (!srv) return fail(SPASM_EINVAL, "server is NULL");
    hipStream_t sa = srv->st;
    // 1. admission in arrival order; the prefix runs on the admission stream
    std::vector<int> admitted;
    while (!srv->pending.empty()) {
        int si = -1;
        for (size_t i = 0; i < srv->slots.size(); ++i)
            if (!srv->slots[i].used) {
                si = (int)i;
                break;
            }
        if (si < 0) break;
        const Request &r = srv->pending.front();
        const size_t need = request_footprint(r.prob, r.cfg);
        size_t off = 0;
        if (!srv->alloc(need, &off)) break;
        Slot &s = srv->slots[(size_t)si];
        s.used = true;
        s.ready = false;
        s.r = r;
        s.off = off;
        s.bytes = need;
        s.L = solve_layout(r.prob->kp, r.cfg);
        s.opt_off = off + align256(s.L.total);
        s.k_done = 0;
        s.steps = 0;
        s.finishing = false;
        srv->pending.pop_front();
        int rc = enqueue_prefix(s.r.prob, s.r.cfg, srv->arena + s.off, s.L, sa);
        if (rc) return rc;
        SPASM_HIP(launch_zero(srv->arena + s.opt_off, opt_bytes(s.r.prob, s.r.cfg), sa));
        s.ready = true;
        s.fresh = true;
        admitted.push_back(si);
    }
    // 2. one batched launch per class of ready solves, each class on its own stream, with
    //    a chunk of iterations sized from the class's measured time per iteration
    //    (solves admitted in this step form their own launches on the admission stream,
    //    right behind their prefix, so a request that finds the server idle starts at once)
    std::map<ClassKey, std::vector<int>> classes, fresh;
    for (size_t i = 0; i < srv->slots.size(); ++i) {
        const Slot &s = srv->slots[i];
        if (s.used && s.ready)
            (s.fresh ? fresh : classes)[{traj_threads(s.r.prob->kp.B, s.r.cfg.W), s.r.prob->kp.chunk}].push_back((int)i);
    }
    double slowest = 0.0;
    for (auto *group : {&classes, &fresh})
        for (auto &cl : *group) {
            auto it = srv->ms_per_iter.find(cl.first);
            if (it != srv->ms_per_iter.end()) slowest = std::max(slowest, it->second);
        }
    // 0 until some class has been timed; otherwise the slowest class's iters_per_step
    // iterations, and at least MIN_STEP_MS of work
    const double step_ms = slowest > 0.0 ? std::max(slowest * srv->iters, MIN_STEP_MS) : 0.0;
    struct Launch {
        ClassKey key;
        int stream, event, iters;
    };
    std::vector<Launch> launches;
    int nd = 0, li = 0;
    std::vector<std::pair<ClassKey, std::vector<int>>> order;
    for (auto &cl : fresh) order.push_back(cl);
    for (auto &cl : classes) order.push_back(cl);
    const size_t n_fresh = fresh.size();
    for (size_t oi = 0; oi < order.size(); ++oi) {
        auto &cl = order[oi];
        const bool is_fresh = oi < n_fresh;
        int chunk = srv->iters;
        auto it = srv->ms_per_iter.find(cl.first);
        if (step_ms > 0.0 && it != srv->ms_per_iter.end() && it->second > 0.0)
            chunk = (int)std::max(1.0, std::min(64.0 * srv->iters, std::floor(step_ms / it->second + 1e-6)));
        const int d0 = nd;
        int first = 0, most = 0;
        for (int i : cl.second) {
            Slot &s = srv->slots[(size_t)i];
            const spasm_solve_config &c = s.r.cfg;
            const int k1 = std::min(c.K, s.k_done + chunk);
            most = std::max(most, k1 - s.k_done);
            s.finishing = k1 == c.K;
            s.k_next = k1;
            ServeSolve &d = srv->h_desc[nd++];
            std::memset(&d, 0, sizeof(d));
            d.P = s.r.prob->kp;
            char *w = srv->arena + s.off;
            TrajArgs &a = d.a;
            a.P = c.M;
            a.W = c.W;
            a.q_in = (const float *)(w + s.L.q);
            a.q_out = (float *)(w + s.L.q);
            a.pose_in = (const float *)(w + s.L.pose);
            a.pose_out = (float *)(w + s.L.pose);
            a.opt = (float *)(srv->arena + s.opt_off);
            a.k_begin = s.k_done + 1;
            a.k_end = k1 + 1;
            a.k_lin2 = (int)std::lround(s.r.prob->lin_frac2 * c.K);
            a.cost = s.finishing ? (float *)(w + s.L.c2) : nullptr;
            a.viol = s.finishing ? (float *)(w + s.L.v2) : nullptr;
            d.first = first;
            first += c.M;
        }
        const int sidx = is_fresh ? -1 : li % N_CLASS_STREAMS, eidx = li < MAX_CLASS_LAUNCHES ? li : -1;
        hipStream_t cst = is_fresh ? sa : srv->cs[sidx];
        SPASM_HIP(hipMemcpyAsync(srv->d_desc + d0, srv->h_desc + d0, sizeof(ServeSolve) * (size_t)(nd - d0),
                                 hipMemcpyHostToDevice, cst));
        if (eidx >= 0) SPASM_HIP(hipEventRecord(srv->ev[2 * eidx], cst));
        SPASM_HIP(launch_serve(cl.first.second, cl.first.first, first, srv->d_desc + d0, nd - d0, cst));
        if (eidx >= 0) SPASM_HIP(hipEventRecord(srv->ev[2 * eidx + 1], cst));
        launches.push_back({cl.first, sidx, eidx, most});
        // 3. finish the solves of this class that reached K, on the same stream
        for (int i : cl.second) {
            Slot &s = srv->slots[(size_t)i];
            if (!s.finishing) continue;
            char *w = srv->arena + s.off;
            int rc = enqueue_finish(s.r.prob, s.r.cfg, w, s.L, s.r.best_q, s.r.best_pose, cst);
            if (rc) return rc;
            SPASM_HIP(hipMemcpyAsync(srv->h_info + 8 * i, w + s.L.info, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, cst));
            SPASM_HIP(hipMemcpyAsync(srv->h_finfo + 4 * i, w + s.L.finfo, 4 * sizeof(float), hipMemcpyDeviceToHost,
                                     cst));
        }
        ++li;
    }
    SPASM_HIP(hipStreamSynchronize(sa));
    for (int i = 0; i < N_CLASS_STREAMS; ++i) SPASM_HIP(hipStreamSynchronize(srv->cs[i]));
    // measured time per iteration of each class (exponentially smoothed)
    for (const Launch &l : launches) {
        if (l.event < 0 || l.iters <= 0) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, srv->ev[2 * l.event], srv->ev[2 * l.event + 1]) != hipSuccess) continue;
        const double per = ms / l.iters;
        auto it = srv->ms_per_iter.find(l.key);
        if (it == srv->ms_per_iter.end())
            srv->ms_per_iter[l.key] = per;
        else
            it->second = 0.5 * it->second + 0.5 * per;
    }
    // 4. retire
    int active = 0;
    for (size_t i = 0; i < srv->slots.size(); ++i) {
        Slot &s = srv->slots[i];
        if (!s.used) continue;
        s.steps++;
        s.fresh = false;
        s.k_done = s.k_next;
        if (!s.finishing) {
            ++active;
            continue;
        }
        spasm_completion c;
        std::memset(&c, 0, sizeof(c));
        c.req_id = s.r.req_id;
        c.status = SPASM_OK;
        c.steps = s.steps;
        const int32_t *info = srv->h_info + 8 * i;
        const float *finfo = srv->h_finfo + 4 * i;
        c.result.stage1_sat = info[0];
        c.result.rounds = info[1];
        c.result.n_sat = info[2];
        c.result.best = info[3];
        c.result.success = info[2] > 0;
        c.result.viol = finfo[0];
        c.result.cost = finfo[1];
        c.result.length = finfo[2];
        srv->done.push_back(c);
        srv->release(s.off, s.bytes);
        s.used = false;
        s.ready = false;
        s.fresh = false;
        s.finishing = false;
    }
    if (n_active) *n_active = active;
    if (n_pending) *n_pending = (int32_t)srv->pending.size();
    return SPASM_OK;
}

extern "C" int spasm_server_poll(spasm_server srv, spasm_completion *out, int32_t max, int32_t *n_out)
{
    if (!srv || !n_out || (max > 0 && !out)) return fail(SPASM_EINVAL, "bad arguments");
    int n = 0;
    while (n < max && !srv->done.empty()) {
        out[n++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_out = n;
    return SPASM_OK;
}

extern "C" void spasm_server_destroy(spasm_server srv)
{
    if (!srv) return;
    srv->cleanup();
    delete srv;
}
