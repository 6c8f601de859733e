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
    int32_t end_status = 0;      // nonzero: no further rounds; the request ends with
                                 // this status once its rounds in flight end
                                 // (WSX_ECANCELED, or WSX_EHIP after a failed launch)
    bool inject_fail = false;    // test hook: its next launch is reported failed
    hipEvent_t done_ev = nullptr;
    int group = -1;
    Clock::time_point t_submit, t_admit, t_done;
};

// One issued round of a group: its launch table and the (request, steps) it
// covers. A group keeps up to kSlots rounds queued on its stream, so the next
// round is on the device before the current one ends.
constexpr int kSlots = 2;
struct Round {
    hipEvent_t ev = nullptr;
    bool inflight = false;
    std::vector<std::pair<int64_t, int32_t>> members;
    Segment* host_table = nullptr;   // pinned
    Segment* dev_table = nullptr;    // in the arena
};

struct Group {
    int kind = 0;
    wsx_policy policy{};
    hipStream_t stream = nullptr;
    Round round[kSlots];
    std::deque<int> order;   // slots in flight, oldest first (stream order)
    int next = 0;            // the slot the next round uses
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
    for (int k = 0; k < kSlots; ++k) {
        Round& rd = g.round[k];
        if (hipEventCreateWithFlags(&rd.ev, hipEventDisableTiming) != hipSuccess) return -1;
        if (hipHostMalloc((void**)&rd.host_table, sizeof(Segment) * S->desc.max_batch) !=
            hipSuccess)
            return -1;
        // launch tables sit at the start of the arena, reserved at creation
        rd.dev_table = reinterpret_cast<Segment*>(
            S->arena_base +
            align256(sizeof(Segment) * S->desc.max_batch) * (S->groups.size() * kSlots + k));
    }
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

// A round's member, or nullptr if the caller has released it: a request that
// completed in a round is marked done by its own event, recorded before the
// round's, so it can be released while the round's event is still pending.
Request* member(wsx_server* S, int64_t id) {
    auto it = S->requests.find(id);
    return it == S->requests.end() ? nullptr : it->second.get();
}

void fail_round(wsx_server* S, Round& rd, int code) {
    for (auto& m : rd.members) {
        Request* r = member(S, m.first);
        if (r && r->status == 1) fail_request(S, r, code);
    }
    rd.members.clear();
    rd.inflight = false;
    S->cv_done.notify_all();
}

// The returns of a request whose last round was just enqueued, right behind
// it on the group's stream, and the event that marks the request complete.
void issue_returns(wsx_server* S, Request* r, hipStream_t stream) {
    hipError_t e = launch_returns(r->traj.reward, r->traj.value, r->traj.done,
                                  r->traj.last_value, r->req.horizon, r->rows, r->req.gamma,
                                  r->req.lambda, 1, r->ret, r->adv, 0, stream);
    if (e == hipSuccess && !r->done_ev) e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->done_ev, stream);
    r->returns_issued = true;
    if (e != hipSuccess) {
        fail_request(S, r, WSX_EHIP);
        S->cv_done.notify_all();
    }
}

// The segment of request r's next `steps` steps (advances its counters).
Segment next_segment(wsx_server* S, Request* r, int32_t steps, int32_t tile_begin) {
    wsx_env* env = S->sessions[r->session].env;
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
    sg.tile_begin = tile_begin;
    sg.last = r->issued + steps == r->req.horizon ? 1 : 0;   // V(s_T) once, at the end
    env->step += (uint32_t)steps;
    r->issued += steps;
    return sg;
}

// Issues, per group with a free slot, one round covering the next chunk of
// every admitted request of the group (up to max_batch), as one fused launch.
// If that launch fails, each member is launched on its own so that only the
// request whose launch fails is failed.
bool launch_rounds(wsx_server* S) {
    bool any = false;
    for (size_t gi = 0; gi < S->groups.size(); ++gi) {
        Group& g = S->groups[gi];
        if ((int)g.order.size() >= kSlots) continue;
        std::vector<Request*> batch;
        for (auto& kv : S->requests) {
            Request* r = kv.second.get();
            if (r->status == 1 && r->group == (int)gi && r->issued < r->req.horizon &&
                r->end_status == 0)
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
        const int slot = g.next;
        Round& rd = g.round[slot];
        int32_t tiles = 0;
        bool injected = false;
        std::vector<std::pair<Request*, int32_t>> plan;
        for (size_t i = 0; i < batch.size(); ++i) {
            Request* r = batch[i];
            const int32_t steps = std::min(S->desc.chunk_steps, r->req.horizon - r->issued);
            plan.push_back({r, steps});
            injected |= r->inject_fail;
            rd.host_table[i] = next_segment(S, r, steps, tiles);
            tiles += S->sessions[r->session].env->n_tiles;
        }
        const wsx_env* env0 = S->sessions[batch[0]->session].env;
        const int per_cu = fused_blocks_per_cu(v);
        hipError_t e = hipMemcpyAsync(rd.dev_table, rd.host_table, sizeof(Segment) * batch.size(),
                                      hipMemcpyHostToDevice, g.stream);
        if (e == hipSuccess && !injected) {
            Batch b{};
            b.table = rd.dev_table;
            b.n_segs = (int32_t)batch.size();
            b.n_tiles = tiles;
            e = launch_fused(v, b, std::max(1, std::min(tiles, env0->cus * per_cu)), g.stream);
            if (e == hipSuccess) S->st.launches++;
        }
        rd.members.clear();
        if (e != hipSuccess || injected) {
            // one launch per member (inline segment): only a member whose own
            // launch fails is failed
            for (size_t i = 0; i < plan.size(); ++i) {
                Request* r = plan[i].first;
                Segment sg = rd.host_table[i];
                sg.tile_begin = 0;
                const int32_t n_tiles = S->sessions[r->session].env->n_tiles;
                hipError_t ei = hipSuccess;
                if (r->inject_fail) {
                    r->inject_fail = false;
                    ei = hipErrorLaunchFailure;
                } else {
                    Batch b{};
                    b.inl[0] = sg;
                    b.n_segs = 1;
                    b.n_tiles = n_tiles;
                    ei = launch_fused(v, b, std::max(1, std::min(n_tiles, env0->cus * per_cu)),
                                      g.stream);
                }
                if (ei != hipSuccess) {
                    // its earlier rounds may still be writing its memory: it
                    // ends when they have (poll), without these steps
                    r->issued -= plan[i].second;
                    S->sessions[r->session].env->step -= (uint32_t)plan[i].second;
                    r->end_status = WSX_EHIP;
                    continue;
                }
                S->st.launches++;
                rd.members.push_back({r->id, plan[i].second});
            }
        } else {
            for (auto& [r, steps] : plan) rd.members.push_back({r->id, steps});
        }
        // the returns of the requests this round completes, right behind it
        for (auto& m : rd.members) {
            Request* r = member(S, m.first);
            if (r && r->status == 1 && r->issued == r->req.horizon) issue_returns(S, r, g.stream);
        }
        e = hipEventRecord(rd.ev, g.stream);
        rd.inflight = true;
        g.order.push_back(slot);
        g.next = (slot + 1) % kSlots;
        if (e != hipSuccess) fail_round(S, rd, WSX_EHIP);
        any = true;
    }
    return any;
}

bool poll(wsx_server* S) {
    bool any = false;
    for (auto& g : S->groups) {
        // rounds complete in stream order: look at the oldest first
        while (!g.order.empty()) {
            Round& rd = g.round[g.order.front()];
            const hipError_t q = hipEventQuery(rd.ev);
            if (q == hipErrorNotReady) break;
            g.order.pop_front();
            any = true;
            if (q != hipSuccess) {
                fail_round(S, rd, WSX_EHIP);
                continue;
            }
            for (auto& m : rd.members)
                if (Request* r = member(S, m.first)) r->finished += m.second;
            rd.members.clear();
            rd.inflight = false;
        }
    }
    for (auto& kv : S->requests) {
        Request* r = kv.second.get();
        if (r->status != 1) continue;
        if (r->end_status != 0 && !r->returns_issued && r->finished == r->issued) {
            // a cancelled (or failed) request ends once its rounds in flight
            // have ended
            r->status = r->end_status;
            r->t_done = Clock::now();
            S->sessions[r->session].busy = false;
            any = true;
            S->cv_done.notify_all();
            continue;
        }
        if (!r->returns_issued || !r->done_ev) continue;
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
        if (!g.order.empty()) return true;
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
            for (auto& g : S->groups) inflight |= !g.order.empty();
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
                // device work in flight: poll again at once (a sleep of a few
                // microseconds lasts tens on a loaded host); the next round of
                // every group is already queued behind the current one
                lk.unlock();
                std::this_thread::yield();
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
    const size_t reserve = align256(sizeof(Segment) * desc->max_batch) * kMaxGroups * kSlots;
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
                            align256(sizeof(Segment) * S->desc.max_batch) * kMaxGroups * kSlots;
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

int wsx_server_cancel(wsx_server* S, int64_t id) {
    if (!S) return fail(WSX_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->requests.find(id);
    if (it == S->requests.end()) return fail(WSX_EINVAL, "no request %lld", (long long)id);
    Request* r = it->second.get();
    if (r->status == 0) {
        S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), id), S->queue.end());
        r->status = WSX_ECANCELED;
        r->t_done = Clock::now();
        S->cv_done.notify_all();
        return WSX_OK;
    }
    if (r->status != 1 || r->returns_issued)
        return fail(WSX_ESTATE, "request %lld has already ended or is completing", (long long)id);
    if (r->end_status == 0) r->end_status = WSX_ECANCELED;
    S->cv_work.notify_one();
    return WSX_OK;
}

int wsx_server_inject_launch_failure(wsx_server* S, int64_t id) {
    if (!S) return fail(WSX_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->requests.find(id);
    if (it == S->requests.end()) return fail(WSX_EINVAL, "no request %lld", (long long)id);
    if (it->second->status > 1 || it->second->status < 0)
        return fail(WSX_ESTATE, "request %lld has ended", (long long)id);
    it->second->inject_fail = true;
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
        for (auto& rd : g.round) {
            (void)hipEventDestroy(rd.ev);
            (void)hipHostFree(rd.host_table);
        }
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
