// abi.cpp -- the C ABI declared in include/wsx.h: argument validation, the
// environment handle (state-block layout, market tile table, step counter),
// variant selection and the launch of the roll-out, reset and returns
// kernels. No C++ exception leaves this file.
#include "../../include/wsx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace wsx;

namespace wsx {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(WSX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Shapes of each kind and the default tile (rows, waves) of its fused kernel.
bool kind_info(int kind, KindInfo& k) {
    switch (kind) {
    case WSX_CARTPOLE: k = {4, 4, 2, WSX_F32, 64, 16, 4, 1}; return true;
    case WSX_PENDULUM: k = {2, 3, 0, WSX_BF16, 256, 80, 8, 2}; return true;
    case WSX_ACROBOT: k = {4, 6, 0, WSX_BF16, 256, 80, 8, 2}; return true;
    case WSX_MARKET: k = {32, 32, 50, WSX_BF16, 256, 128, 4, 1}; return true;
    case WSX_REACTION: k = {21, 20, 40, WSX_FP8_E4M3, 512, 16, 8, 2}; return true;
    }
    return user_kind_info(kind, k);
}

int n_head_of(const KindInfo& k) { return (k.nact ? k.nact : 1) + 1; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout_of(const KindInfo& k, int64_t n_envs, int64_t n_rows, bool market, bool reaction) {
    Layout L{};
    size_t at = 0;
    L.state = at;
    at = align256(at + (size_t)k.sd * n_rows * 4);
    L.obs = at;
    at = align256(at + (size_t)k.od * n_rows * 4);
    L.head = at;
    at = align256(at + (size_t)n_head_of(k) * n_rows * 4);
    L.offsets = at;
    if (market) at = align256(at + (size_t)(n_envs + 1) * 4);
    L.tiles = at;
    if (market) at = align256(at + (size_t)n_envs * sizeof(Tile));
    L.row_map = at;
    if (market) at = align256(at + (size_t)n_rows * 4);
    L.slot_map = at;
    if (market) at = align256(at + (size_t)n_rows);
    L.cache = at;   // the reaction's FP64 energy terms [NCACHE][n_rows]
    if (reaction) at = align256(at + (size_t)kReactionCache * n_rows * 8);
    L.step = at;   // [step counter, epoch] for graph replays
    at = align256(at + 8);
    L.total = at;
    return L;
}

// The compiled kernel with the fewest row slots that holds tiles of
// `tile_rows` rows; waves / occupancy 0 match any compiled value (the first
// listed wins among kernels of the same row capacity).
static bool find_any(int kind, int kind2, int dtype, int hidden, int waves, int tile_rows,
                     int occupancy, Variant& out) {
    if (kind >= kUserKindBase || kind2 >= kUserKindBase) {   // one compiled shape per user kind
        Variant v;
        if (kind2 != 0 || !user_variant(kind, v)) return false;
        if (v.dtype != dtype || v.hidden != hidden || tile_rows < 1 || v.tile_rows < tile_rows ||
            (waves != 0 && v.waves != waves) || (occupancy != 0 && v.occupancy != occupancy))
            return false;
        out = v;
        return true;
    }
    bool found = false;
    for (int i = 0; i < n_variants(); ++i) {
        const Variant& v = variant(i);
        const bool kinds = kind2 == 0 ? (v.kind == kind && v.kind2 == 0)
                                      : ((v.kind == kind && v.kind2 == kind2) ||
                                         (v.kind == kind2 && v.kind2 == kind));
        if (kinds && v.dtype == dtype && v.hidden == hidden && tile_rows >= 1 &&
            v.tile_rows >= tile_rows && (waves == 0 || v.waves == waves) &&
            (occupancy == 0 || v.occupancy == occupancy) &&
            (!found || v.tile_rows < out.tile_rows)) {
            out = v;
            found = true;
        }
    }
    return found;
}

bool find_variant(int kind, int dtype, int hidden, int waves, int tile_rows, int occupancy,
                  Variant& out) {
    return find_any(kind, 0, dtype, hidden, waves, tile_rows, occupancy, out);
}

bool find_pair_variant(int kind, int kind2, int dtype, int hidden, int waves, int tile_rows,
                       int occupancy, Variant& out) {
    return find_any(kind, kind2, dtype, hidden, waves, tile_rows, occupancy, out);
}

}  // namespace wsx

EnvArgs wsx::env_args(const wsx_env* env) {
    EnvArgs a{};
    a.kind = env->kind;
    a.state = reinterpret_cast<float*>(env->block + env->lay.state);
    a.obs_scratch = reinterpret_cast<float*>(env->block + env->lay.obs);
    a.head_scratch = reinterpret_cast<float*>(env->block + env->lay.head);
    a.params = env->params;
    a.offsets = env->kind == WSX_MARKET ? reinterpret_cast<const int32_t*>(env->block + env->lay.offsets)
                                        : nullptr;
    a.tiles = env->kind == WSX_MARKET ? reinterpret_cast<const Tile*>(env->block + env->lay.tiles)
                                      : nullptr;
    a.row_map = env->kind == WSX_MARKET
                    ? reinterpret_cast<const int32_t*>(env->block + env->lay.row_map)
                    : nullptr;
    a.slot_map = env->kind == WSX_MARKET
                     ? reinterpret_cast<const uint8_t*>(env->block + env->lay.slot_map)
                     : nullptr;
    a.cache = env->kind == WSX_REACTION ? reinterpret_cast<double*>(env->block + env->lay.cache)
                                        : nullptr;
    a.step_ptr = nullptr;
    a.n_rows = env->n_rows;
    a.n_envs = (int32_t)env->n_envs;
    a.n_tiles = env->n_tiles;
    a.tile_rows = env->tile_rows;
    a.k0 = (uint32_t)(env->seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(env->seed >> 32);
    a.epoch = env->epoch;
    a.t0 = env->step;
    return a;
}

TrajArgs wsx::traj_at(const TrajArgs& t, const KindInfo& k, size_t slots) {
    TrajArgs o = t;
    o.obs = t.obs + slots * (size_t)k.od;
    o.action = static_cast<char*>(t.action) + slots * (k.nact ? 1 : 4);
    o.reward = t.reward + slots;
    o.done = t.done + slots;
    o.value = t.value + slots;
    o.logp = t.logp + slots;
    return o;
}

int wsx::check_traj(const wsx_env* env, const wsx_traj* traj, int32_t horizon) {
    if (horizon < 0) return fail(WSX_EINVAL, "horizon must be >= 0");
    if (!traj) return fail(WSX_EINVAL, "traj is NULL");
    if (traj->capacity < horizon)
        return fail(WSX_EINVAL, "traj capacity %d < horizon %d", traj->capacity, horizon);
    if (!traj->last_value || (horizon > 0 && (!traj->obs || !traj->action || !traj->reward ||
                                              !traj->done || !traj->value || !traj->logp)))
        return fail(WSX_EINVAL, "trajectory pointer is NULL");
    if ((uint64_t)env->step + (uint64_t)horizon > 0xFFFFFFFFull)
        return fail(WSX_EINVAL, "step counter would wrap");
    return WSX_OK;
}

TrajArgs wsx::traj_args(const wsx_traj* traj) {
    TrajArgs ta{};
    ta.obs = traj->obs;
    ta.action = traj->action;
    ta.reward = traj->reward;
    ta.done = traj->done;
    ta.value = traj->value;
    ta.logp = traj->logp;
    ta.last_value = traj->last_value;
    return ta;
}

int wsx::check_policy(const wsx_policy* p, const KindInfo& k, int kind) {
    if (!p) return fail(WSX_EINVAL, "policy is NULL");
    if (p->dtype != k.dtype)
        return fail(WSX_EUNSUPPORTED, "kind %d runs dtype %d policies (got %d)", kind, k.dtype, p->dtype);
    if (p->d_in != k.od) return fail(WSX_EINVAL, "policy d_in %d != observation size %d", p->d_in, k.od);
    if (p->h1 != k.hidden || p->h2 != k.hidden)
        return fail(WSX_EUNSUPPORTED, "kind %d runs %d-unit hidden layers (got %d, %d)", kind,
                    k.hidden, p->h1, p->h2);
    if (p->n_head != n_head_of(k))
        return fail(WSX_EINVAL, "policy n_head %d != %d", p->n_head, n_head_of(k));
    if (!p->w1 || !p->w2 || !p->w3 || !p->b1 || !p->b2 || !p->b3)
        return fail(WSX_EINVAL, "policy weight or bias pointer is NULL");
    if (p->dtype == WSX_FP8_E4M3) {
        if (!p->s1 || !p->s2 || !p->s3) return fail(WSX_EINVAL, "FP8 policy needs row scales");
        for (int i = 0; i < 3; ++i) {
            int ex;
            const float m = frexpf(p->act_scale[i], &ex);
            if (!(p->act_scale[i] > 0.0f) || m != 0.5f)
                return fail(WSX_EINVAL, "act_scale[%d] must be a positive power of two", i);
        }
    }
    if (k.nact == 0 && !p->log_std) return fail(WSX_EINVAL, "continuous policy needs log_std");
    return WSX_OK;
}

PolicyArgs wsx::policy_args(const wsx_policy* p) {
    PolicyArgs a{};
    a.w1 = p->w1;
    a.w2 = p->w2;
    a.w3 = p->w3;
    a.b1 = p->b1;
    a.b2 = p->b2;
    a.b3 = p->b3;
    a.s1 = p->s1;
    a.s2 = p->s2;
    a.s3 = p->s3;
    a.log_std = p->log_std;
    for (int i = 0; i < 3; ++i) a.act_scale[i] = p->act_scale[i];
    a.d_in = p->d_in;
    a.hidden = p->h1;
    a.n_head = p->n_head;
    return a;
}

// Whole market envs into tiles of at most `cap` agents by first-fit
// decreasing (envs by agent count, largest first, each into the first tile
// with room; ties in env order), so the tiles are nearly full: the kernel's
// time per tile does not depend on its fill, only the number of tiles does.
// Within a tile the envs keep ascending env order and each env's agents stay
// together; the row map lists the tiles' rows in tile order, the slot map
// each row's env index within its tile.
void wsx::pack_market_tiles(const int32_t* off, int64_t n_envs, int cap, std::vector<Tile>& tiles,
                            std::vector<int32_t>& row_map, std::vector<uint8_t>& slot_map) {
    std::vector<int32_t> order((size_t)n_envs);
    for (int64_t e = 0; e < n_envs; ++e) order[(size_t)e] = (int32_t)e;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return off[a + 1] - off[a] > off[b + 1] - off[b];
    });
    std::vector<int> room;                        // free agent slots of each tile
    std::vector<std::vector<int32_t>> members;    // envs of each tile
    for (const int32_t e : order) {
        const int c = off[e + 1] - off[e];
        size_t t = 0;
        while (t < room.size() && room[t] < c) ++t;
        if (t == room.size()) {
            room.push_back(cap);
            members.emplace_back();
        }
        room[t] -= c;
        members[t].push_back(e);
    }
    tiles.clear();
    row_map.clear();
    slot_map.clear();
    row_map.reserve((size_t)off[n_envs]);
    slot_map.reserve((size_t)off[n_envs]);
    for (auto& m : members) {
        std::sort(m.begin(), m.end());
        Tile tl{(int32_t)row_map.size(), 0, 0, (int32_t)m.size()};
        for (size_t i = 0; i < m.size(); ++i)
            for (int32_t r = off[m[i]]; r < off[m[i] + 1]; ++r) {
                row_map.push_back(r);
                slot_map.push_back((uint8_t)i);
            }
        tl.row1 = (int32_t)row_map.size();
        tiles.push_back(tl);
    }
}

extern "C" {

const char* wsx_last_error(void) { return g_last_error.c_str(); }

int wsx_env_state_bytes(int32_t kind, int64_t n_envs, int64_t n_rows, size_t* bytes) {
    KindInfo k;
    if (!kind_info(kind, k)) return fail(WSX_EINVAL, "unknown environment kind %d", kind);
    if (n_envs <= 0 || n_rows < n_envs) return fail(WSX_EINVAL, "need 0 < n_envs <= n_rows");
    if (kind != WSX_MARKET && n_rows != n_envs)
        return fail(WSX_EINVAL, "single-agent kinds have n_rows == n_envs");
    if (n_rows > 0x7FFFFFFF) return fail(WSX_EUNSUPPORTED, "at most 2^31-1 rows");
    if (!bytes) return fail(WSX_EINVAL, "bytes is NULL");
    *bytes = layout_of(k, n_envs, n_rows, kind == WSX_MARKET, kind == WSX_REACTION).total;
    return WSX_OK;
}

int wsx_env_create(const wsx_env_desc* d, wsx_env** out) {
    if (!d || !out) return fail(WSX_EINVAL, "desc and out must not be NULL");
    *out = nullptr;
    KindInfo k;
    if (!kind_info(d->kind, k)) return fail(WSX_EINVAL, "unknown environment kind %d", d->kind);
    if (d->n_envs <= 0 || d->n_envs > 0x7FFFFFFF) return fail(WSX_EINVAL, "n_envs out of range");
    if (!d->state) return fail(WSX_EINVAL, "state block is NULL");
    const bool market = d->kind == WSX_MARKET;
    if (market != (d->agent_offsets != nullptr))
        return fail(WSX_EINVAL, "agent_offsets is required for the market and only for it");
    if ((d->kind == WSX_REACTION) != (d->params != nullptr))
        return fail(WSX_EINVAL, "params is required for the reaction walk and only for it");
    if (d->occupancy < 0 || d->tile_rows < 0 || d->waves < 0)
        return fail(WSX_EINVAL, "tile_rows, waves and occupancy must be >= 0");
    const bool deflt = !d->tile_rows && !d->waves && !d->occupancy;
    if (market && d->agent_offsets[0] != 0) return fail(WSX_EINVAL, "agent_offsets[0] must be 0");
    // the autotuner's shape for this set on this device, if it has tuned it
    int device = 0, cus = 0;
    wsx_tune_entry tuned{};
    const bool use_tuned =
        deflt && hipGetDevice(&device) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        tune_lookup(d->kind, d->n_envs, market ? d->agent_offsets[d->n_envs] : d->n_envs, cus,
                    tuned);
    const int tile_rows = use_tuned ? tuned.tile_rows : d->tile_rows ? d->tile_rows : k.tile_rows;
    const int waves = use_tuned ? tuned.waves : d->waves ? d->waves : (deflt ? k.waves : 0);
    const int occupancy =
        use_tuned ? tuned.occupancy : d->occupancy ? d->occupancy : (deflt ? k.occupancy : 0);
    Variant probe;
    if (!find_variant(d->kind, k.dtype, k.hidden, waves, tile_rows, occupancy, probe))
        return fail(WSX_EUNSUPPORTED,
                    "no compiled kernel with %d rows per tile, %d waves, occupancy %d for kind %d",
                    tile_rows, waves, occupancy, d->kind);

    int64_t n_rows = d->n_envs;
    std::vector<Tile> tiles;
    std::vector<int32_t> row_map;
    std::vector<uint8_t> slot_map;
    if (market) {
        const int32_t* off = d->agent_offsets;
        for (int64_t e = 0; e < d->n_envs; ++e) {
            const int64_t c = (int64_t)off[e + 1] - off[e];
            if (c < 1 || c > tile_rows)
                return fail(WSX_EINVAL, "env %lld has %lld agents (allowed 1..%d)", (long long)e,
                            (long long)c, tile_rows);
        }
        n_rows = off[d->n_envs];
        pack_market_tiles(off, d->n_envs, tile_rows, tiles, row_map, slot_map);
    }
    wsx_env* env = new (std::nothrow) wsx_env();
    if (!env) return fail(WSX_EINVAL, "out of host memory");
    env->kind = d->kind;
    env->info = k;
    env->n_envs = d->n_envs;
    env->n_rows = n_rows;
    env->seed = d->seed;
    env->step = 0;
    env->epoch = 0;
    env->block = static_cast<char*>(d->state);
    env->params = d->params;
    env->lay = layout_of(k, d->n_envs, n_rows, market, d->kind == WSX_REACTION);
    env->tile_rows = tile_rows;
    env->waves = probe.waves;
    env->occupancy = probe.occupancy;
    env->n_tiles = market ? (int)tiles.size() : (int)((n_rows + tile_rows - 1) / tile_rows);
    env->chunk = use_tuned ? tuned.chunk_steps : 0;
    env->graph = nullptr;
    env->capture_stream = nullptr;
    hipError_t e = hipGetDevice(&env->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&env->cus, hipDeviceAttributeMultiprocessorCount, env->device);
    if (e == hipSuccess && market) {
        e = hipMemcpy(env->block + env->lay.offsets, d->agent_offsets,
                      (size_t)(d->n_envs + 1) * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(env->block + env->lay.tiles, tiles.data(), tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(env->block + env->lay.row_map, row_map.data(), row_map.size() * 4,
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(env->block + env->lay.slot_map, slot_map.data(), slot_map.size(),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        delete env;
        return hip_fail(e, "wsx_env_create");
    }
    *out = env;
    return WSX_OK;
}

int wsx_env_destroy(wsx_env* env) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    if (env->graph) (void)hipGraphExecDestroy(env->graph);
    if (env->capture_stream) (void)hipStreamDestroy(env->capture_stream);
    delete env;
    return WSX_OK;
}

int wsx_env_tiles(const wsx_env* env, int32_t* n_tiles, int32_t* capacity) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    if (n_tiles) *n_tiles = env->n_tiles;
    if (capacity) *capacity = env->tile_rows;
    return WSX_OK;
}

int wsx_env_info(const wsx_env* env, int64_t* n_rows, uint32_t* step, uint32_t* epoch) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    if (n_rows) *n_rows = env->n_rows;
    if (step) *step = env->step;
    if (epoch) *epoch = env->epoch;
    return WSX_OK;
}

int wsx_env_set_step(wsx_env* env, uint32_t step) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    env->step = step;
    return WSX_OK;
}

int wsx_env_shape(const wsx_env* env, int32_t* tile_rows, int32_t* waves, int32_t* occupancy,
                  int32_t* chunk_steps) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    if (tile_rows) *tile_rows = env->tile_rows;
    if (waves) *waves = env->waves;
    if (occupancy) *occupancy = env->occupancy;
    if (chunk_steps) *chunk_steps = env->chunk;
    return WSX_OK;
}

int wsx_env_set_chunk(wsx_env* env, int32_t chunk_steps) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    if (chunk_steps < 0) return fail(WSX_EINVAL, "chunk_steps must be >= 0");
    env->chunk = chunk_steps;
    return WSX_OK;
}


int wsx_env_reset(wsx_env* env, uint32_t epoch, void* stream) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    env->epoch = epoch;
    env->step = 0;
    const hipError_t e = launch_reset(env->kind, env_args(env), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_env_reset");
    return WSX_OK;
}



int wsx_rollout(wsx_env* env, const wsx_policy* policy, int32_t horizon, const wsx_traj* traj,
                int32_t mode, void* stream) {
    if (!env) return fail(WSX_EINVAL, "env is NULL");
    int rc = check_policy(policy, env->info, env->kind);
    if (rc) return rc;
    rc = check_traj(env, traj, horizon);
    if (rc) return rc;
    Variant v;
    if (!find_variant(env->kind, policy->dtype, policy->h1, env->waves, env->tile_rows,
                      env->occupancy, v))
        return fail(WSX_EUNSUPPORTED, "no compiled kernel for this policy and tile");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const EnvArgs ea = env_args(env);
    const PolicyArgs pa = policy_args(policy);
    const TrajArgs ta = traj_args(traj);
    hipError_t e = hipSuccess;
    const int grid = std::max(1, std::min(env->n_tiles, env->cus * fused_blocks_per_cu(v)));
    // fused launch of `steps` steps from trajectory slot `first`
    auto fused = [&](const EnvArgs& a, int first, int steps, bool last, hipStream_t st) {
        Batch b{};
        b.table = nullptr;
        Segment& sg = b.inl[0];
        sg.env = a;
        sg.env.t0 += (uint32_t)first;
        sg.tr = traj_at(ta, env->info, (size_t)first * (size_t)env->n_rows);
        sg.tr.last_value = ta.last_value;
        sg.pol = pa;
        sg.steps = steps;
        sg.tile_begin = 0;
        sg.last = last ? 1 : 0;
        b.n_segs = 1;
        b.n_tiles = env->n_tiles;
        return launch_fused(v, b, grid, st);
    };
    if (env->kind >= kUserKindBase && (mode == WSX_MODE_PLAIN || mode == WSX_MODE_GRAPH))
        return fail(WSX_EUNSUPPORTED, "user kinds run the fused modes only");
    if (mode == WSX_MODE_FUSED) {
        e = fused(ea, 0, horizon, true, s);
    } else if (mode == WSX_MODE_PLAIN) {
        e = launch_plain(v, ea, pa, ta, horizon, false, s);
    } else if (mode == WSX_MODE_GRAPH || mode == WSX_MODE_FUSED_GRAPH) {
        // the launches read the step counter and the epoch from the state
        // block, so one captured graph serves every call with the same
        // buffers and horizon
        EnvArgs ga = ea;
        ga.step_ptr = reinterpret_cast<const uint32_t*>(env->block + env->lay.step);
        ga.t0 = 0;
        const int chunk = mode == WSX_MODE_GRAPH ? 0 : env->chunk;
        const int desc[3] = {horizon, mode, chunk};
        std::vector<char> key(sizeof(PolicyArgs) + sizeof(TrajArgs) + sizeof desc + sizeof(Variant));
        std::memcpy(key.data(), &pa, sizeof pa);
        std::memcpy(key.data() + sizeof pa, &ta, sizeof ta);
        std::memcpy(key.data() + sizeof pa + sizeof ta, desc, sizeof desc);
        std::memcpy(key.data() + sizeof pa + sizeof ta + sizeof desc, &v, sizeof v);
        if (!env->graph || env->graph_key != key) {
            if (env->graph) {
                (void)hipGraphExecDestroy(env->graph);
                env->graph = nullptr;
            }
            if (!env->capture_stream) {
                e = hipStreamCreateWithFlags(&env->capture_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(e, "wsx_rollout (capture stream)");
            }
            e = hipStreamBeginCapture(env->capture_stream, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return hip_fail(e, "wsx_rollout (begin capture)");
            hipError_t le = hipSuccess;
            if (mode == WSX_MODE_GRAPH) {
                le = launch_plain(v, ga, pa, ta, horizon, true, env->capture_stream);
            } else {
                const int c = chunk > 0 ? chunk : std::max(horizon, 1);
                int first = 0;
                do {
                    const int steps = std::min(c, horizon - first);
                    le = fused(ga, first, steps, first + steps == horizon, env->capture_stream);
                    first += steps;
                } while (le == hipSuccess && first < horizon);
            }
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(env->capture_stream, &g);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) e = hipGraphInstantiate(&env->graph, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e, "wsx_rollout (capture)");
            env->graph_key = key;
        }
        e = launch_set_step(const_cast<uint32_t*>(ga.step_ptr), env->step, env->epoch, s);
        if (e == hipSuccess) e = hipGraphLaunch(env->graph, s);
    } else {
        return fail(WSX_EINVAL, "unknown mode %d", mode);
    }
    if (e != hipSuccess) return hip_fail(e, "wsx_rollout");
    env->step += (uint32_t)horizon;
    return WSX_OK;
}

int wsx_rollout_batch(wsx_env* const* envs, const wsx_policy* const* policies,
                      const wsx_traj* const* trajs, int32_t n, int32_t horizon, void* stream) {
    return wsx_rollout_batch_ext(envs, policies, trajs, n, horizon, nullptr, stream);
}

int wsx_rollout_batch_ext(wsx_env* const* envs, const wsx_policy* const* policies,
                          const wsx_traj* const* trajs, int32_t n, int32_t horizon,
                          const wsx_rollout_ext* ext, void* stream) {
    if (!envs || !policies || !trajs) return fail(WSX_EINVAL, "envs, policies, trajs must not be NULL");
    const bool gae = ext && ext->returns;
    if (gae) {
        if (!ext->ret || !ext->adv) return fail(WSX_EINVAL, "ext->ret and ext->adv must not be NULL");
        if (ext->out_dtype != WSX_F32 && ext->out_dtype != WSX_F64)
            return fail(WSX_EUNSUPPORTED, "returns are written as WSX_F32 or WSX_F64");
        if (!(ext->gamma >= 0.0 && ext->gamma <= 1.0) || !(ext->lambda >= 0.0 && ext->lambda <= 1.0))
            return fail(WSX_EINVAL, "gamma and lambda must lie in [0, 1]");
    }
    if (n < 1 || n > kInlineSegments)
        return fail(WSX_EINVAL, "a batch holds 1 to %d environment sets (got %d)", kInlineSegments, n);
    int kinds[2] = {0, 0}, n_kinds = 0, tile_max = 0;
    for (int i = 0; i < n; ++i) {
        if (!envs[i]) return fail(WSX_EINVAL, "envs[%d] is NULL", i);
        int rc = check_policy(policies[i], envs[i]->info, envs[i]->kind);
        if (rc) return rc;
        rc = check_traj(envs[i], trajs[i], horizon);
        if (rc) return rc;
        for (int j = 0; j < i; ++j)
            if (envs[j] == envs[i]) return fail(WSX_EINVAL, "envs[%d] repeats envs[%d]", i, j);
        if (policies[i]->dtype != policies[0]->dtype || policies[i]->h1 != policies[0]->h1)
            return fail(WSX_EUNSUPPORTED, "the policies of a batch share dtype and width");
        if (envs[i]->device != envs[0]->device)
            return fail(WSX_EINVAL, "the sets of a batch live on one device");
        const int k = envs[i]->kind;
        if (!(n_kinds > 0 && kinds[0] == k) && !(n_kinds > 1 && kinds[1] == k)) {
            if (n_kinds == 2) return fail(WSX_EUNSUPPORTED, "a batch mixes at most two kinds");
            kinds[n_kinds++] = k;
        }
        tile_max = std::max(tile_max, envs[i]->tile_rows);
    }
    Variant v;
    const bool ok = n_kinds == 1
                        ? find_variant(kinds[0], policies[0]->dtype, policies[0]->h1,
                                       envs[0]->waves, tile_max, envs[0]->occupancy, v)
                        : find_pair_variant(kinds[0], kinds[1], policies[0]->dtype,
                                            policies[0]->h1, envs[0]->waves, tile_max,
                                            envs[0]->occupancy, v);
    if (!ok)
        return fail(WSX_EUNSUPPORTED,
                    "no fused kernel for kinds %d/%d with %d waves, occupancy %d, %d-row tiles",
                    kinds[0], kinds[1], envs[0]->waves, envs[0]->occupancy, tile_max);
    if (gae)
        for (int i = 0; i < n; ++i)
            if (horizon > 0 && (!ext->ret[i] || !ext->adv[i]))
                return fail(WSX_EINVAL, "ext->ret[%d] / ext->adv[%d] is NULL", i, i);
    const bool reset = ext && ext->reset;
    Batch b{};
    b.table = nullptr;
    int tiles = 0;
    for (int i = 0; i < n; ++i) {
        Segment& sg = b.inl[i];
        sg.env = env_args(envs[i]);
        if (reset) {   // the state the reset kernel would leave: step 0 of the epoch
            sg.env.epoch = ext->epoch;
            sg.env.t0 = 0;
        }
        sg.tr = traj_args(trajs[i]);
        sg.pol = policy_args(policies[i]);
        sg.gae = GaeArgs{};
        if (gae && horizon > 0) {
            sg.gae.ret = ext->ret[i];
            sg.gae.adv = ext->adv[i];
            sg.gae.gamma = ext->gamma;
            sg.gae.lambda = ext->lambda;
            sg.gae.bootstrap = ext->bootstrap ? 1 : 0;
            sg.gae.out_f64 = ext->out_dtype == WSX_F64 ? 1 : 0;
        }
        sg.steps = horizon;
        sg.tile_begin = tiles;
        sg.last = 1;
        sg.reset = reset ? 1 : 0;
        tiles += envs[i]->n_tiles;
    }
    b.n_segs = n;
    b.n_tiles = tiles;
    b.any_reset = reset ? 1 : 0;
    b.any_gae = gae && horizon > 0 ? 1 : 0;
    const int grid = std::max(1, std::min(tiles, envs[0]->cus * fused_blocks_per_cu(v)));
    const hipError_t e = launch_fused(v, b, grid, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_rollout_batch");
    for (int i = 0; i < n; ++i) {
        if (reset) {
            envs[i]->epoch = ext->epoch;
            envs[i]->step = 0;
        }
        envs[i]->step += (uint32_t)horizon;
    }
    return WSX_OK;
}

int wsx_compute_returns(const float* reward, const float* value, const uint8_t* done,
                        const float* last_value, int32_t horizon, int64_t rows, double gamma,
                        double lambda, int32_t bootstrap, void* returns, void* advantages,
                        int32_t out_dtype, void* stream) {
    if (horizon < 0 || rows < 0) return fail(WSX_EINVAL, "negative horizon or rows");
    if (out_dtype != WSX_F32 && out_dtype != WSX_F64)
        return fail(WSX_EUNSUPPORTED, "returns are written as WSX_F32 or WSX_F64");
    if (!(gamma >= 0.0 && gamma <= 1.0) || !(lambda >= 0.0 && lambda <= 1.0))
        return fail(WSX_EINVAL, "gamma and lambda must lie in [0, 1]");
    if (horizon == 0 || rows == 0) return WSX_OK;
    if (!reward || !value || !done || !last_value || !returns || !advantages)
        return fail(WSX_EINVAL, "a buffer pointer is NULL");
    const hipError_t e = launch_returns(reward, value, done, last_value, horizon, rows, gamma, lambda,
                                        bootstrap ? 1 : 0, returns, advantages,
                                        out_dtype == WSX_F64 ? 1 : 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_compute_returns");
    return WSX_OK;
}

int wsx_policy_forward(const wsx_policy* policy, const float* obs, int64_t rows, float* head,
                       void* stream) {
    if (!policy) return fail(WSX_EINVAL, "policy is NULL");
    if (rows < 0 || rows > 0x7FFFFFFF) return fail(WSX_EINVAL, "rows out of range");
    // the kind whose policy shape this is
    int kind = 0;
    KindInfo k{};
    for (int c = WSX_CARTPOLE; c <= WSX_REACTION; ++c) {
        KindInfo ki;
        kind_info(c, ki);
        if (ki.dtype == policy->dtype && ki.od == policy->d_in && ki.hidden == policy->h1 &&
            n_head_of(ki) == policy->n_head) {
            kind = c;
            k = ki;
            break;
        }
    }
    if (!kind) return fail(WSX_EUNSUPPORTED, "no compiled kernel for this policy shape");
    int rc = check_policy(policy, k, kind);
    if (rc) return rc;
    if (rows == 0) return WSX_OK;
    if (!obs || !head) return fail(WSX_EINVAL, "obs or head is NULL");
    Variant v;
    if (!find_variant(kind, k.dtype, k.hidden, k.waves, k.tile_rows, k.occupancy, v))
        return fail(WSX_EUNSUPPORTED, "no compiled kernel for this policy shape");
    const hipError_t e = launch_policy_forward(v, policy_args(policy), obs, rows, head,
                                               static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_policy_forward");
    return WSX_OK;
}

int wsx_policy_trace(const wsx_env* env, const wsx_policy* policy, const float* obs,
                     int64_t rows, float* head, void* act1, void* act2, void* stream) {
    if (!env || !policy) return fail(WSX_EINVAL, "env or policy is NULL");
    if (rows < 0 || rows > 0x7FFFFFFF) return fail(WSX_EINVAL, "rows out of range");
    if (env->kind >= kUserKindBase)
        return fail(WSX_EUNSUPPORTED, "no policy trace for user environment kinds");
    int rc = check_policy(policy, env->info, env->kind);
    if (rc) return rc;
    if (rows == 0) return WSX_OK;
    if (!obs || !head || !act1 || !act2) return fail(WSX_EINVAL, "a buffer pointer is NULL");
    Variant v;
    if (!find_variant(env->kind, env->info.dtype, env->info.hidden, env->waves, env->tile_rows,
                      env->occupancy, v))
        return fail(WSX_EUNSUPPORTED, "no compiled kernel for the set's shape");
    const hipError_t e = launch_policy_trace(v, policy_args(policy), obs, rows, head, act1, act2,
                                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_policy_trace");
    return WSX_OK;
}

int wsx_quantize(int32_t dtype, float scale, const float* x, float* y, int64_t n, void* stream) {
    if (dtype != WSX_F32 && dtype != WSX_BF16 && dtype != WSX_FP8_E4M3)
        return fail(WSX_EINVAL, "unknown dtype %d", dtype);
    int ex;
    if (!(scale > 0.0f) || frexpf(scale, &ex) != 0.5f)
        return fail(WSX_EINVAL, "scale must be a positive power of two");
    if (n < 0) return fail(WSX_EINVAL, "n < 0");
    if (n == 0) return WSX_OK;
    if (!x || !y) return fail(WSX_EINVAL, "x or y is NULL");
    const hipError_t e = launch_quantize(dtype, scale, x, y, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_quantize");
    return WSX_OK;
}

// ------------------------------------------------------------- update --
static int ac_grid(int64_t samples) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t tiles = (ac_chunk_samples(samples) + 31) / 32;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cus));
}

static int check_ac_policy(const wsx_policy* p) {
    if (!p) return fail(WSX_EINVAL, "policy is NULL");
    if (p->dtype == WSX_FP8_E4M3)
        return fail(WSX_EUNSUPPORTED, "the update covers FP32 and BF16 policies");
    if (p->dtype != WSX_F32 && p->dtype != WSX_BF16) return fail(WSX_EINVAL, "unknown dtype %d", p->dtype);
    if (p->h1 != p->h2) return fail(WSX_EUNSUPPORTED, "hidden layers of different widths");
    if (p->d_in < 1 || p->n_head < 2) return fail(WSX_EINVAL, "policy d_in < 1 or n_head < 2");
    if (!ac_supported(p->dtype, p->h1, p->d_in, p->n_head))
        return fail(WSX_EUNSUPPORTED, "no update kernel for dtype %d, hidden %d, d_in %d, n_head %d",
                    p->dtype, p->h1, p->d_in, p->n_head);
    if (!p->w1 || !p->w2 || !p->w3 || !p->b1 || !p->b2 || !p->b3)
        return fail(WSX_EINVAL, "policy weight or bias pointer is NULL");
    return WSX_OK;
}

int wsx_ac_grad_workspace_bytes(const wsx_policy* policy, int64_t samples, size_t* bytes) {
    if (const int rc = check_ac_policy(policy)) return rc;
    if (samples < 1) return fail(WSX_EINVAL, "samples must be >= 1");
    if (!bytes) return fail(WSX_EINVAL, "bytes is NULL");
    const int g = ac_grid(samples);
    *bytes = ac_workspace_bytes(policy->dtype, policy->h1, samples, g);
    return WSX_OK;
}

int wsx_ac_grad(const wsx_policy* policy, int32_t n_actions, const float* obs,
                const void* action, const float* returns, const float* advantages,
                int64_t samples, float value_coef, float entropy_coef, const wsx_grads* grads,
                void* workspace, size_t workspace_bytes, void* stream) {
    if (const int rc = check_ac_policy(policy)) return rc;
    if (n_actions == 0) {
        if (policy->n_head != 2)
            return fail(WSX_EUNSUPPORTED, "Gaussian policies with %d action dimensions",
                        policy->n_head - 1);
        if (!policy->log_std) return fail(WSX_EINVAL, "Gaussian policy needs log_std");
    } else if (n_actions < 2 || n_actions > 255 || policy->n_head != n_actions + 1) {
        return fail(WSX_EINVAL, "n_actions %d does not match n_head %d (categorical: 2..255)",
                    n_actions, policy->n_head);
    }
    if (samples < 1) return fail(WSX_EINVAL, "samples must be >= 1");
    if (!obs || !action || !returns || !advantages)
        return fail(WSX_EINVAL, "obs, action, returns or advantages is NULL");
    if (!std::isfinite(value_coef) || !std::isfinite(entropy_coef))
        return fail(WSX_EINVAL, "loss coefficients must be finite");
    if (!grads || !grads->w1 || !grads->b1 || !grads->w2 || !grads->b2 || !grads->w3 ||
        !grads->b3)
        return fail(WSX_EINVAL, "gradient pointer is NULL");
    if (n_actions == 0 && !grads->log_std)
        return fail(WSX_EINVAL, "Gaussian policy: grads->log_std is NULL");
    const int g = ac_grid(samples);
    const size_t need = ac_workspace_bytes(policy->dtype, policy->h1, samples, g);
    if (!workspace || workspace_bytes < need)
        return fail(WSX_EINVAL, "workspace of %zu bytes < %zu needed", workspace_bytes, need);
    AcLaunch l{};
    l.args.pol = policy_args(policy);
    l.args.obs = obs;
    l.args.action = action;
    l.args.ret = returns;
    l.args.adv = advantages;
    l.args.n = samples;
    l.args.n_act = n_actions;
    l.args.value_coef = value_coef;
    l.args.entropy_coef = entropy_coef;
    l.args.inv_n = (float)(1.0 / (double)samples);
    l.dtype = policy->dtype;
    l.workspace = workspace;
    l.grid = g;
    l.out = AcOut{grads->w1, grads->b1, grads->w2, grads->b2, grads->w3, grads->b3,
                  n_actions == 0 ? grads->log_std : nullptr};
    const hipError_t e = launch_ac_grad(l, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_ac_grad");
    return WSX_OK;
}

static_assert(kAcStaticSamples == WSX_AC_STATIC_MAX_SAMPLES, "one sample bound");

int wsx_ac_grad_static(const wsx_policy* policy, int32_t n_actions, const float* obs,
                       const void* action, const float* returns, const float* advantages,
                       int64_t samples, float value_coef, float entropy_coef,
                       const wsx_grads* grads, void* stream) {
    if (samples > WSX_AC_STATIC_MAX_SAMPLES)
        return fail(WSX_EINVAL, "wsx_ac_grad_static takes at most %d samples (got %lld)",
                    WSX_AC_STATIC_MAX_SAMPLES, (long long)samples);
    if (const int rc = check_ac_policy(policy)) return rc;
    if (samples >= 1) {
        const int g = ac_grid(samples);
        if (ac_workspace_bytes(policy->dtype, policy->h1, samples, g) > ac_static_capacity())
            return fail(WSX_EUNSUPPORTED, "the static workspace does not hold this policy shape");
    }
    hipError_t err;
    void* ws = ac_static_workspace(&err);
    if (!ws) return hip_fail(err, "wsx_ac_grad_static: address of the static workspace");
    return wsx_ac_grad(policy, n_actions, obs, action, returns, advantages, samples, value_coef,
                       entropy_coef, grads, ws, ac_static_capacity(), stream);
}

int wsx_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, int32_t step,
                  float lr, float beta1, float beta2, float eps, void* store, int32_t store_dtype,
                  void* stream) {
    if (n < 0) return fail(WSX_EINVAL, "n < 0");
    if (step < 1) return fail(WSX_EINVAL, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(WSX_EINVAL, "betas must lie in [0, 1)");
    if (!std::isfinite(lr) || !(eps >= 0.0f) || !std::isfinite(eps))
        return fail(WSX_EINVAL, "lr must be finite and eps finite and >= 0");
    if (store && store_dtype != WSX_F32 && store_dtype != WSX_BF16)
        return fail(WSX_EINVAL, "store_dtype must be WSX_F32 or WSX_BF16");
    if (n == 0) return WSX_OK;
    if (!param || !grad || !m || !v) return fail(WSX_EINVAL, "param, grad, m or v is NULL");
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    const hipError_t e = launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, c1, c2, store,
                                     store_dtype, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_adam_step");
    return WSX_OK;
}

int wsx_adam_step_many(const wsx_adam_tensor* tensors, int32_t n_tensors, int32_t step, float lr,
                       float beta1, float beta2, float eps, void* stream) {
    if (!tensors) return fail(WSX_EINVAL, "tensors is NULL");
    if (n_tensors < 1 || n_tensors > WSX_ADAM_MAX_TENSORS)
        return fail(WSX_EINVAL, "n_tensors must lie in 1..%d", WSX_ADAM_MAX_TENSORS);
    if (step < 1) return fail(WSX_EINVAL, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(WSX_EINVAL, "betas must lie in [0, 1)");
    if (!std::isfinite(lr) || !(eps >= 0.0f) || !std::isfinite(eps))
        return fail(WSX_EINVAL, "lr must be finite and eps finite and >= 0");
    AdamTable t{};
    int used = 0;
    int64_t most = 0;
    for (int i = 0; i < n_tensors; ++i) {
        const wsx_adam_tensor& a = tensors[i];
        if (a.n < 0) return fail(WSX_EINVAL, "tensor %d: n < 0", i);
        if (a.store && a.store_dtype != WSX_F32 && a.store_dtype != WSX_BF16)
            return fail(WSX_EINVAL, "tensor %d: store_dtype must be WSX_F32 or WSX_BF16", i);
        if (a.n == 0) continue;
        if (!a.param || !a.grad || !a.m || !a.v)
            return fail(WSX_EINVAL, "tensor %d: param, grad, m or v is NULL", i);
        // the ABI's WSX_F32 / WSX_BF16 codes are the kernels' format codes
        t.seg[used++] = AdamSeg{a.param, a.grad, a.m, a.v, a.n, a.store, a.store_dtype};
        most = std::max(most, a.n);
    }
    if (used == 0) return WSX_OK;
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    const hipError_t e = launch_adam_many(t, used, most, lr, beta1, beta2, eps, c1, c2,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "wsx_adam_step_many");
    return WSX_OK;
}

}  // extern "C"
