// serve.cpp -- the roll-out server: continuous batching of roll-out requests
// (C ABI in include/wsx.h).
//
// The paper runs thousands of replicas concurrently on one GPU with roll-out
// data kept in device memory (arXiv 2408.00930, Sec. 2 and App. B). The
// server applies that to a stream of independent requests: a scheduler thread
// admits queued requests when their memory fits the caller's arena (the HBM
// budget), and in every round issues, per (environment kind, policy), one
// fused launch covering the next chunk of every admitted request. A request
// that arrives while others run joins the next round; kinds run concurrently
// on their own streams. Results are independent of the mix: each replica's
// numbers depend only on its own seed, epoch and step counter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "admission.h"
#include "internal.h"
#include "kernels.h"

using namespace wsx;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kMaxGroups = 8;

struct Session {
    wsx_env* env = nullptr;
    size_t off = 0, bytes = 0;
    bool busy = false;
    bool keep = false;
};

struct Request {
    int64_t id = 0;
    wsx_request req{};
    wsx_policy policy{};
    std::vector<int32_t> offsets;
    int32_t status = 0;   // 0 queued, 1 admitted, 2 done, < 0 failed
    int64_t session = 0;
    int64_t rows = 0;
    size_t off = 0, bytes = 0;
    wsx_traj traj{};
    float* ret = nullptr;
    float* adv = nullptr;
    int32_t issued = 0, finished = 0;   // steps launched / completed on the device
    bool returns_issued = false;
    hipEvent_t done_ev = nullptr;
    int group = -1;
    Clock::time_point t_submit, t_admit, t_done;
};

struct Group {
    int kind = 0;
    wsx_policy policy{};
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    bool inflight = false;
    std::vector<std::pair<int64_t, int32_t>> members;   // (request, steps) in flight
    Segment* host_table = nullptr;   // pinned
    Segment* dev_table = nullptr;    // in the arena
};

size_t traj_bytes(const KindInfo& k, int64_t rows, int32_t T) {
    const size_t n = (size_t)rows * (size_t)T;
    size_t b = 0;
    b += align256(n * k.od * 4);              // obs
    b += align256(n * (k.nact ? 1 : 4));      // action
    b += align256(n * 4) * 3;                 // reward, value, logp
    b += align256(n);                         // done
    b += align256((size_t)rows * 4);          // last_value
    b += align256(n * 4) * 2;                 // returns, advantages
    return b;
}

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct wsx_server {
    wsx_server_desc desc{};
    Arena arena;          // offsets into [arena_base, arena_base + arena_bytes)
    char* arena_base = nullptr;
    std::mutex mu;
    std::condition_variable cv_done, cv_work;
    std::thread worker;
    bool stop = false;
    int device = 0;
    std::deque<int64_t> queue;
    std::map<int64_t, std::unique_ptr<Request>> requests;
    std::map<int64_t, Session> sessions;
    std::vector<Group> groups;
    int64_t next_id = 1, next_session = 1;
    wsx_server_stats st{};
};

namespace {

int group_of(wsx_server* S, int kind, const wsx_policy& p) {
    for (size_t i = 0; i < S->groups.size(); ++i)
        if (S->groups[i].kind == kind && std::memcmp(&S->groups[i].policy, &p, sizeof p) == 0)
            return (int)i;
    if ((int)S->groups.size() >= kMaxGroups) return -1;
    Group g;
    g.kind = kind;
    g.policy = p;
    if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess) return -1;
    if (hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess) return -1;
    if (hipHostMalloc((void**)&g.host_table, sizeof(Segment) * S->desc.max_batch) != hipSuccess)
        return -1;
    // launch tables sit at the start of the arena, reserved at creation
    g.dev_table = reinterpret_cast<Segment*>(
        S->arena_base + align256(sizeof(Segment) * S->desc.max_batch) * S->groups.size());
    S->groups.push_back(g);
    return (int)S->groups.size() - 1;
}

void free_session(wsx_server* S, int64_t sid) {
    auto it = S->sessions.find(sid);
    if (it == S->sessions.end()) return;
    if (it->second.env) wsx_env_destroy(it->second.env);
    S->arena.release(it->second.off, it->second.bytes);
    S->sessions.erase(it);
}

// Admit one queued request if its memory fits; false to keep it queued.
bool try_admit(wsx_server* S, Request* r) {
    KindInfo k;
    kind_info(r->req.kind, k);
    const bool fresh = r->req.session == 0;
    if (!fresh) {
        auto it = S->sessions.find(r->req.session);
        if (it == S->sessions.end()) {
            r->status = WSX_EINVAL;
            return true;
        }
        if (it->second.busy) return false;
        r->rows = it->second.env->n_rows;
    } else {
        r->rows = r->req.kind == WSX_MARKET ? r->offsets.back() : r->req.n_envs;
    }
    const int g = group_of(S, r->req.kind, r->policy);
    if (g < 0) return false;
    const size_t tb = traj_bytes(k, r->rows, r->req.horizon);
    size_t toff = 0, soff = 0, sbytes = 0;
    if (fresh) {
        if (wsx_env_state_bytes(r->req.kind, r->req.n_envs, r->rows, &sbytes) != WSX_OK) {
            r->status = WSX_EINVAL;
            return true;
        }
        if (!S->arena.alloc(sbytes, &soff)) return false;
    }
    if (!S->arena.alloc(tb, &toff)) {
        if (fresh) S->arena.release(soff, sbytes);
        return false;
    }
    int64_t sid = r->req.session;
    if (fresh) {
        wsx_env_desc d{};
        d.kind = r->req.kind;
        // every session of a kind runs the kind's built-in kernel shape (not
        // an autotuner entry for its size), so that one launch covers them all
        d.tile_rows = k.tile_rows;
        d.waves = k.waves;
        d.occupancy = k.occupancy;
        d.n_envs = r->req.n_envs;
        d.seed = r->req.seed;
        d.state = S->arena_base + soff;
        d.agent_offsets = r->req.kind == WSX_MARKET ? r->offsets.data() : nullptr;
        d.params = r->req.params;
        wsx_env* env = nullptr;
        int rc = wsx_env_create(&d, &env);
        if (rc == WSX_OK) rc = wsx_env_reset(env, r->req.epoch, S->groups[g].stream);
        if (rc != WSX_OK) {
            if (env) wsx_env_destroy(env);
            S->arena.release(soff, sbytes);
            S->arena.release(toff, tb);
            r->status = rc;
            return true;
        }
        sid = S->next_session++;
        Session s;
        s.env = env;
        s.off = soff;
        s.bytes = sbytes;
        s.keep = r->req.keep_session != 0;
        S->sessions[sid] = s;
    }
    Session& sess = S->sessions[sid];
    sess.busy = true;
    if (!fresh && !r->req.keep_session) sess.keep = false;
    r->session = sid;
    r->group = g;
    r->off = toff;
    r->bytes = tb;
    // carve the trajectory and the returns out of the block
    const size_t n = (size_t)r->rows * (size_t)r->req.horizon;
    char* p = S->arena_base + toff;
    auto take = [&p](size_t bytes) {
        char* q = p;
        p += align256(bytes);
        return q;
    };
    r->traj.capacity = r->req.horizon;
    r->traj.obs = reinterpret_cast<float*>(take(n * k.od * 4));
    r->traj.action = take(n * (k.nact ? 1 : 4));
    r->traj.reward = reinterpret_cast<float*>(take(n * 4));
    r->traj.value = reinterpret_cast<float*>(take(n * 4));
    r->traj.logp = reinterpret_cast<float*>(take(n * 4));
    r->traj.done = reinterpret_cast<uint8_t*>(take(n));
    r->traj.last_value = reinterpret_cast<float*>(take((size_t)r->rows * 4));
    r->ret = reinterpret_cast<float*>(take(n * 4));
    r->adv = reinterpret_cast<float*>(take(n * 4));
    r->status = 1;
    r->t_admit = Clock::now();
    S->st.admitted++;
    return true;
}

bool admit(wsx_server* S) {
    const auto now = Clock::now();
    return admit_in_order(
        S->queue, 100.0,
        [&](int64_t id) {
            Request* r = S->requests[id].get();
            if (!try_admit(S, r)) return false;
            if (r->status < 0) {
                r->t_done = Clock::now();
                S->cv_done.notify_all();
            }
            return true;
        },
        [&](int64_t id) { return ms_between(S->requests[id]->t_submit, now); });
}

void fail_request(wsx_server* S, Request* r, int code) {
    r->status = code;
    r->t_done = Clock::now();
    S->sessions[r->session].busy = false;
}

void fail_group(wsx_server* S, Group& g, int code) {
    for (auto& m : g.members) fail_request(S, S->requests[m.first].get(), code);
    g.members.clear();
    g.inflight = false;
    S->cv_done.notify_all();
}

bool launch_rounds(wsx_server* S) {
    bool any = false;
    for (size_t gi = 0; gi < S->groups.size(); ++gi) {
        Group& g = S->groups[gi];
        if (g.inflight) continue;
        std::vector<Request*> batch;
        for (auto& kv : S->requests) {
            Request* r = kv.second.get();
            if (r->status == 1 && r->group == (int)gi && r->issued < r->req.horizon)
                batch.push_back(r);
            if ((int)batch.size() == S->desc.max_batch) break;
        }
        if (batch.empty()) continue;
        // one kernel for the round: the waves and occupancy the sessions share
        // and the row capacity of the tallest tile among them
        const wsx_env* first = S->sessions[batch[0]->session].env;
        int tile_max = 0;
        for (Request* r : batch) tile_max = std::max(tile_max, S->sessions[r->session].env->tile_rows);
        Variant v{};
        if (!find_variant(first->kind, batch[0]->policy.dtype, batch[0]->policy.h1, first->waves,
                          tile_max, first->occupancy, v)) {
            for (Request* r : batch) fail_request(S, r, WSX_EUNSUPPORTED);
            S->cv_done.notify_all();
            continue;
        }
        int32_t tiles = 0;
        for (size_t i = 0; i < batch.size(); ++i) {
            Request* r = batch[i];
            wsx_env* env = S->sessions[r->session].env;
            const int32_t steps = std::min(S->desc.chunk_steps, r->req.horizon - r->issued);
            const size_t base = (size_t)r->issued * (size_t)r->rows;
            Segment sg{};
            sg.env = env_args(env);
            sg.tr.obs = r->traj.obs + base * env->info.od;
            sg.tr.action = static_cast<char*>(r->traj.action) + base * (env->info.nact ? 1 : 4);
            sg.tr.reward = r->traj.reward + base;
            sg.tr.done = r->traj.done + base;
            sg.tr.value = r->traj.value + base;
            sg.tr.logp = r->traj.logp + base;
            sg.tr.last_value = r->traj.last_value;
            sg.pol = policy_args(&r->policy);
            sg.steps = steps;
            sg.tile_begin = tiles;
            sg.last = r->issued + steps == r->req.horizon ? 1 : 0;   // V(s_T) once, at the end
            tiles += env->n_tiles;
            g.host_table[i] = sg;
            env->step += (uint32_t)steps;
            r->issued += steps;
            g.members.push_back({r->id, steps});
        }
        hipError_t e = hipMemcpyAsync(g.dev_table, g.host_table, sizeof(Segment) * batch.size(),
                                      hipMemcpyHostToDevice, g.stream);
        Batch b{};
        b.table = g.dev_table;
        b.n_segs = (int32_t)batch.size();
        b.n_tiles = tiles;
        const wsx_env* env0 = S->sessions[batch[0]->session].env;
        const int grid = std::max(1, std::min(tiles, env0->cus * fused_blocks_per_cu(v)));
        if (e == hipSuccess) e = launch_fused(v, b, grid, g.stream);
        if (e == hipSuccess) e = hipEventRecord(g.ev, g.stream);
        g.inflight = true;
        if (e != hipSuccess) {
            fail_group(S, g, WSX_EHIP);
            continue;
        }
        S->st.launches++;
        any = true;
    }
    return any;
}

bool poll(wsx_server* S) {
    bool any = false;
    for (auto& g : S->groups) {
        if (!g.inflight) continue;
        const hipError_t q = hipEventQuery(g.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            fail_group(S, g, WSX_EHIP);
            continue;
        }
        for (auto& m : g.members) {
            Request* r = S->requests[m.first].get();
            r->finished += m.second;
            if (r->finished == r->req.horizon && !r->returns_issued) {
                hipError_t e = launch_returns(r->traj.reward, r->traj.value, r->traj.done,
                                              r->traj.last_value, r->req.horizon, r->rows,
                                              r->req.gamma, r->req.lambda, 1, r->ret, r->adv, 0,
                                              g.stream);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(r->done_ev, g.stream);
                r->returns_issued = true;
                if (e != hipSuccess) {
                    fail_request(S, r, WSX_EHIP);
                    S->cv_done.notify_all();
                }
            }
        }
        g.members.clear();
        g.inflight = false;
        any = true;
    }
    for (auto& kv : S->requests) {
        Request* r = kv.second.get();
        if (r->status != 1 || !r->returns_issued || !r->done_ev) continue;
        const hipError_t q = hipEventQuery(r->done_ev);
        if (q == hipErrorNotReady) continue;
        r->status = q == hipSuccess ? 2 : WSX_EHIP;
        r->t_done = Clock::now();
        S->sessions[r->session].busy = false;
        if (r->status == 2) {
            S->st.completed++;
            S->st.env_steps += S->sessions[r->session].env->n_envs * (int64_t)r->req.horizon;
        }
        any = true;
        S->cv_done.notify_all();
    }
    return any;
}

bool busy(const wsx_server* S) {
    for (const auto& g : S->groups)
        if (g.inflight) return true;
    for (const auto& kv : S->requests)
        if (kv.second->status == 1) return true;
    return false;
}

void worker_loop(wsx_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stop) {
            // cancel what is still queued; finish the device work in flight
            for (int64_t id : S->queue) S->requests[id]->status = WSX_ESTATE;
            S->queue.clear();
            for (auto& kv : S->requests)
                if (kv.second->status == 1 && kv.second->issued == kv.second->finished &&
                    !kv.second->returns_issued)
                    kv.second->status = WSX_ESTATE;
            S->cv_done.notify_all();
            bool inflight = false;
            for (auto& g : S->groups) inflight |= g.inflight;
            for (auto& kv : S->requests)
                inflight |= kv.second->status == 1 && kv.second->returns_issued;
            if (!inflight) break;
        }
        bool progressed = false;
        if (!S->stop) progressed |= admit(S);
        if (!S->stop) progressed |= launch_rounds(S);
        progressed |= poll(S);
        if (!progressed) {
            if (busy(S)) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }
}

void fill_result(const wsx_server* S, const Request* r, wsx_result* out) {
    std::memset(out, 0, sizeof *out);
    out->status = r->status;
    out->session = r->session;
    out->n_rows = r->rows;
    if (r->status >= 1) {
        out->traj = r->traj;
        out->returns = r->ret;
        out->advantages = r->adv;
        out->queue_ms = ms_between(r->t_submit, r->t_admit);
    }
    if (r->status == 2) out->latency_ms = ms_between(r->t_submit, r->t_done);
    (void)S;
}

}  // namespace

extern "C" {

int wsx_server_create(const wsx_server_desc* desc, wsx_server** out) {
    if (!desc || !out) return fail(WSX_EINVAL, "desc and out must not be NULL");
    *out = nullptr;
    if (!desc->arena || desc->arena_bytes == 0) return fail(WSX_EINVAL, "arena is empty");
    if (desc->chunk_steps <= 0 || desc->max_batch <= 0 || desc->max_batch > 4096)
        return fail(WSX_EINVAL, "chunk_steps and max_batch must be positive (max_batch <= 4096)");
    const size_t reserve = align256(sizeof(Segment) * desc->max_batch) * kMaxGroups;
    if (desc->arena_bytes <= reserve) return fail(WSX_EINVAL, "arena smaller than the launch tables");
    wsx_server* S = new (std::nothrow) wsx_server();
    if (!S) return fail(WSX_EINVAL, "out of host memory");
    S->desc = *desc;
    S->arena_base = static_cast<char*>(desc->arena);
    S->arena.init(desc->arena_bytes);
    size_t off;
    S->arena.alloc(reserve, &off);   // the launch tables of up to kMaxGroups groups
    const hipError_t e = hipGetDevice(&S->device);
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "wsx_server_create");
    }
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return WSX_OK;
}

int wsx_server_submit(wsx_server* S, const wsx_request* q, int64_t* id) {
    if (!S || !q || !id) return fail(WSX_EINVAL, "server, request and id must not be NULL");
    KindInfo k;
    if (!kind_info(q->kind, k)) return fail(WSX_EINVAL, "unknown environment kind %d", q->kind);
    if (q->horizon <= 0) return fail(WSX_EINVAL, "horizon must be > 0");
    int rc = check_policy(q->policy, k, q->kind);
    if (rc) return rc;
    if (!(q->gamma >= 0.0 && q->gamma <= 1.0) || !(q->lambda >= 0.0 && q->lambda <= 1.0))
        return fail(WSX_EINVAL, "gamma and lambda must lie in [0, 1]");
    auto r = std::make_unique<Request>();
    r->req = *q;
    r->policy = *q->policy;
    r->req.policy = nullptr;
    int64_t rows = q->n_envs;
    std::lock_guard<std::mutex> lk(S->mu);
    if (q->session == 0) {
        if (q->n_envs <= 0 || q->n_envs > 0x7FFFFFFF) return fail(WSX_EINVAL, "n_envs out of range");
        if ((q->kind == WSX_MARKET) != (q->agent_offsets != nullptr))
            return fail(WSX_EINVAL, "agent_offsets is required for the market and only for it");
        if ((q->kind == WSX_REACTION) != (q->params != nullptr))
            return fail(WSX_EINVAL, "params is required for the reaction walk and only for it");
        if (q->kind == WSX_MARKET) {
            r->offsets.assign(q->agent_offsets, q->agent_offsets + q->n_envs + 1);
            if (r->offsets[0] != 0) return fail(WSX_EINVAL, "agent_offsets[0] must be 0");
            for (int64_t e = 0; e < q->n_envs; ++e) {
                const int64_t c = (int64_t)r->offsets[e + 1] - r->offsets[e];
                if (c < 1 || c > k.tile_rows)
                    return fail(WSX_EINVAL, "env %lld has %lld agents (allowed 1..%d)",
                                (long long)e, (long long)c, k.tile_rows);
            }
            rows = r->offsets.back();
        }
        size_t sbytes = 0;
        rc = wsx_env_state_bytes(q->kind, q->n_envs, rows, &sbytes);
        if (rc) return rc;
        const size_t need = align256(sbytes) + traj_bytes(k, rows, q->horizon) +
                            align256(sizeof(Segment) * S->desc.max_batch) * kMaxGroups;
        if (need > S->desc.arena_bytes)
            return fail(WSX_EINVAL, "request needs %zu bytes, more than the arena", need);
    } else {
        auto it = S->sessions.find(q->session);
        if (it == S->sessions.end()) return fail(WSX_EINVAL, "no session %lld", (long long)q->session);
        if (it->second.env->kind != q->kind) return fail(WSX_EINVAL, "session is of another kind");
        rows = it->second.env->n_rows;
        const size_t need = traj_bytes(k, rows, q->horizon);
        if (need > S->desc.arena_bytes) return fail(WSX_EINVAL, "request larger than the arena");
    }
    if (S->stop) return fail(WSX_ESTATE, "server is stopping");
    r->id = S->next_id++;
    r->t_submit = Clock::now();
    *id = r->id;
    S->queue.push_back(r->id);
    S->requests[r->id] = std::move(r);
    S->st.submitted++;
    S->cv_work.notify_one();
    return WSX_OK;
}

int wsx_server_wait(wsx_server* S, int64_t id, int32_t timeout_ms, wsx_result* out) {
    if (!S || !out) return fail(WSX_EINVAL, "server and out must not be NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->requests.find(id);
    if (it == S->requests.end()) return fail(WSX_EINVAL, "no request %lld", (long long)id);
    Request* r = it->second.get();
    auto ready = [r] { return r->status == 2 || r->status < 0; };
    if (timeout_ms < 0)
        S->cv_done.wait(lk, ready);
    else
        S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    fill_result(S, r, out);
    if (r->status < 0) return fail(r->status, "request %lld failed", (long long)id);
    if (r->status != 2) return fail(WSX_ETIMEOUT, "request %lld not complete", (long long)id);
    return WSX_OK;
}

int wsx_server_release(wsx_server* S, int64_t id) {
    if (!S) return fail(WSX_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->requests.find(id);
    if (it == S->requests.end()) return fail(WSX_EINVAL, "no request %lld", (long long)id);
    Request* r = it->second.get();
    if (r->status == 0 || r->status == 1) return fail(WSX_ESTATE, "request %lld is still running", (long long)id);
    if (r->bytes) S->arena.release(r->off, r->bytes);
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
    auto s = S->sessions.find(r->session);
    if (s != S->sessions.end() && !s->second.keep && !s->second.busy) free_session(S, r->session);
    S->requests.erase(it);
    return WSX_OK;
}

int wsx_server_close_session(wsx_server* S, int64_t session) {
    if (!S) return fail(WSX_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(session);
    if (it == S->sessions.end()) return fail(WSX_EINVAL, "no session %lld", (long long)session);
    if (it->second.busy) return fail(WSX_ESTATE, "session %lld is in use", (long long)session);
    free_session(S, session);
    return WSX_OK;
}

int wsx_server_get_stats(wsx_server* S, wsx_server_stats* out) {
    if (!S || !out) return fail(WSX_EINVAL, "server and out must not be NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->arena_in_use = S->arena.in_use();
    out->arena_peak = S->arena.peak();
    out->queued = (int32_t)S->queue.size();
    int32_t running = 0;
    for (auto& kv : S->requests) running += kv.second->status == 1;
    out->running = running;
    return WSX_OK;
}

int wsx_server_destroy(wsx_server* S) {
    if (!S) return fail(WSX_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    S->worker.join();
    for (auto& g : S->groups) {
        (void)hipStreamSynchronize(g.stream);
        (void)hipStreamDestroy(g.stream);
        (void)hipEventDestroy(g.ev);
        (void)hipHostFree(g.host_table);
    }
    for (auto& kv : S->requests)
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
    std::vector<int64_t> sids;
    for (auto& kv : S->sessions) sids.push_back(kv.first);
    for (int64_t sid : sids) free_session(S, sid);
    delete S;
    return WSX_OK;
}

}  // extern "C"
