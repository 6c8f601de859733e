// tune.cpp -- the autotuner of the fused roll-out and its process-wide table
// (wsx_autotune, wsx_tune_*): candidate kernel shapes, event timing on the
// caller's stream, text persistence. No C++ exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/wsx.h"
#include "internal.h"
#include "kernels.h"

using namespace wsx;

namespace {

struct Key {
    int32_t kind;
    int64_t n_envs, n_rows;
    int32_t cus;
    bool operator==(const Key& o) const {
        return kind == o.kind && n_envs == o.n_envs && n_rows == o.n_rows && cus == o.cus;
    }
};

struct Row {
    Key key;
    wsx_tune_entry e;
};

std::mutex g_mu;
std::vector<Row> g_table;

void put(std::vector<Row>& t, const Row& r) {
    for (Row& x : t)
        if (x.key == r.key) {
            x = r;
            return;
        }
    t.push_back(r);
}

// Trial buffers carved from the workspace.
struct Trial {
    size_t state_bytes = 0, total = 0;
    size_t off[7] = {};   // obs action reward done value logp last_value
};

Trial trial_layout(const KindInfo& k, int kind, int64_t n_envs, int64_t n_rows, int32_t horizon) {
    Trial t;
    t.state_bytes = layout_of(k, n_envs, n_rows, kind == WSX_MARKET, kind == WSX_REACTION).total;
    size_t at = align256(t.state_bytes);
    const size_t slots = (size_t)horizon * (size_t)n_rows;
    const size_t sizes[7] = {slots * (size_t)k.od * 4, slots * (k.nact ? 1 : 4), slots * 4, slots,
                             slots * 4, slots * 4, (size_t)n_rows * 4};
    for (int i = 0; i < 7; ++i) {
        t.off[i] = at;
        at = align256(at + sizes[i]);
    }
    t.total = at;
    return t;
}

int64_t rows_of(const wsx_env_desc* d) {
    if (d->kind == WSX_MARKET && d->agent_offsets) return d->agent_offsets[d->n_envs];
    return d->n_envs;
}

}  // namespace

bool wsx::tune_lookup(int32_t kind, int64_t n_envs, int64_t n_rows, int32_t cus,
                      wsx_tune_entry& out) {
    std::lock_guard<std::mutex> lk(g_mu);
    const Key k{kind, n_envs, n_rows, cus};
    for (const Row& r : g_table)
        if (r.key == k) {
            out = r.e;
            return true;
        }
    return false;
}

extern "C" {

int wsx_autotune_workspace_bytes(const wsx_env_desc* d, int32_t horizon, size_t* bytes) {
    if (!d || !bytes) return fail(WSX_EINVAL, "desc and bytes must not be NULL");
    KindInfo k;
    if (!kind_info(d->kind, k)) return fail(WSX_EINVAL, "unknown environment kind %d", d->kind);
    if (horizon < 1) return fail(WSX_EINVAL, "horizon must be >= 1");
    if (d->n_envs <= 0 || d->n_envs > 0x7FFFFFFF) return fail(WSX_EINVAL, "n_envs out of range");
    if ((d->kind == WSX_MARKET) != (d->agent_offsets != nullptr))
        return fail(WSX_EINVAL, "agent_offsets is required for the market and only for it");
    *bytes = trial_layout(k, d->kind, d->n_envs, rows_of(d), horizon).total;
    return WSX_OK;
}

int wsx_autotune(const wsx_env_desc* d, const wsx_policy* policy, int32_t horizon, int32_t reps,
                 void* workspace, size_t workspace_bytes, wsx_tune_entry* best, void* stream) {
    size_t need = 0;
    int rc = wsx_autotune_workspace_bytes(d, horizon, &need);
    if (rc) return rc;
    if (!policy) return fail(WSX_EINVAL, "policy is NULL");
    if (reps < 1) return fail(WSX_EINVAL, "reps must be >= 1");
    if (!workspace || workspace_bytes < need)
        return fail(WSX_EINVAL, "workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    KindInfo k;
    kind_info(d->kind, k);
    if (policy->dtype != k.dtype || policy->h1 != k.hidden)
        return fail(WSX_EUNSUPPORTED, "no compiled kernel for this policy");
    const int64_t n_rows = rows_of(d);
    const Trial T = trial_layout(k, d->kind, d->n_envs, n_rows, horizon);
    char* ws = static_cast<char*>(workspace);
    wsx_traj tr{};
    tr.capacity = horizon;
    tr.obs = reinterpret_cast<float*>(ws + T.off[0]);
    tr.action = ws + T.off[1];
    tr.reward = reinterpret_cast<float*>(ws + T.off[2]);
    tr.done = reinterpret_cast<uint8_t*>(ws + T.off[3]);
    tr.value = reinterpret_cast<float*>(ws + T.off[4]);
    tr.logp = reinterpret_cast<float*>(ws + T.off[5]);
    tr.last_value = reinterpret_cast<float*>(ws + T.off[6]);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "wsx_autotune");

    // candidate shapes: every compiled kernel for the policy at its full row
    // capacity, plus the tile heights that deal the rows out evenly over the
    // compute units (one to eight tiles per CU) that the kernel can hold
    struct Cand {
        int tile_rows, waves, occupancy;
    };
    std::vector<Cand> cands;
    auto add = [&](int t, const Variant& v) {
        for (const Cand& c : cands)
            if (c.tile_rows == t && c.waves == v.waves && c.occupancy == v.occupancy) return;
        Variant w;   // the kernel this height runs on must be v itself
        if (find_variant(d->kind, k.dtype, k.hidden, v.waves, t, v.occupancy, w) &&
            w.tile_rows == v.tile_rows)
            cands.push_back({t, v.waves, v.occupancy});
    };
    const bool market = d->kind == WSX_MARKET;
    int max_agents = 1;
    if (market)
        for (int64_t i = 0; i < d->n_envs; ++i)
            max_agents = std::max<int>(max_agents, d->agent_offsets[i + 1] - d->agent_offsets[i]);
    for (int i = 0; i < n_variants(); ++i) {
        const Variant& v = variant(i);
        if (v.kind != d->kind || v.kind2 != 0 || v.dtype != k.dtype || v.hidden != k.hidden)
            continue;
        if (market && v.tile_rows < max_agents) continue;
        add(v.tile_rows, v);
        if (!market)
            for (int per = 1; per <= 8; ++per) {
                const int t = (int)((n_rows + (int64_t)per * cus - 1) / ((int64_t)per * cus));
                if (t >= 1 && t <= v.tile_rows) add(t, v);
            }
    }
    if (cands.empty()) return fail(WSX_EUNSUPPORTED, "no compiled kernel for this policy");

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e != hipSuccess) return hip_fail(e, "wsx_autotune (events)");

    // median time of `reps` roll-outs of the set after one untimed one
    auto measure = [&](const Cand& c, int mode, int chunk, double& ms) -> int {
        wsx_env_desc dd = *d;
        dd.state = ws;
        dd.tile_rows = c.tile_rows;
        dd.waves = c.waves;
        dd.occupancy = c.occupancy;
        wsx_env* env = nullptr;
        int r = wsx_env_create(&dd, &env);
        if (r) return r;
        r = wsx_env_set_chunk(env, chunk);
        if (!r) r = wsx_env_reset(env, 0, stream);
        if (!r) r = wsx_rollout(env, policy, horizon, &tr, mode, stream);
        std::vector<float> t;
        for (int i = 0; !r && i < reps; ++i) {
            hipError_t he = hipEventRecord(ev0, s);
            if (he == hipSuccess && (r = wsx_rollout(env, policy, horizon, &tr, mode, stream)) == 0)
                he = hipEventRecord(ev1, s);
            if (he == hipSuccess && !r) he = hipEventSynchronize(ev1);
            float m = 0.0f;
            if (he == hipSuccess && !r) he = hipEventElapsedTime(&m, ev0, ev1);
            if (he != hipSuccess && !r) r = hip_fail(he, "wsx_autotune (timing)");
            t.push_back(m);
        }
        wsx_env_destroy(env);
        if (r) return r;
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return WSX_OK;
    };

    wsx_tune_entry win{};
    double win_ms = 0.0;
    for (const Cand& c : cands) {
        double ms = 0.0;
        rc = measure(c, WSX_MODE_FUSED, 0, ms);
        if (rc) break;
        if (win_ms == 0.0 || ms < win_ms) {
            win_ms = ms;
            win = {c.tile_rows, c.waves, c.occupancy, 0, 0.0};
        }
    }
    // chunk length of the graph mode for the winning shape: one launch for the
    // whole horizon, or launches of a half, a quarter, an eighth of it
    if (!rc) {
        const Cand w{win.tile_rows, win.waves, win.occupancy};
        double graph_best = 0.0;
        for (int div : {1, 2, 4, 8}) {
            const int chunk = div == 1 ? 0 : (horizon + div - 1) / div;
            if (div > 1 && chunk < 1) break;
            double ms = 0.0;
            rc = measure(w, WSX_MODE_FUSED_GRAPH, chunk, ms);
            if (rc) break;
            if (graph_best == 0.0 || ms < graph_best) {
                graph_best = ms;
                win.chunk_steps = chunk;
            }
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc) return rc;
    win.us_per_step = win_ms * 1000.0 / horizon;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        put(g_table, Row{Key{d->kind, d->n_envs, n_rows, cus}, win});
    }
    if (best) *best = win;
    return WSX_OK;
}

int wsx_autotune_batch_workspace_bytes(const wsx_env_desc* const* descs, int32_t n,
                                       int32_t horizon, size_t* bytes) {
    if (!descs || !bytes) return fail(WSX_EINVAL, "descs and bytes must not be NULL");
    if (n < 1 || n > kInlineSegments)
        return fail(WSX_EINVAL, "a batch holds 1 to %d environment sets", kInlineSegments);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        size_t b = 0;
        if (!descs[i]) return fail(WSX_EINVAL, "descs[%d] is NULL", i);
        const int rc = wsx_autotune_workspace_bytes(descs[i], horizon, &b);
        if (rc) return rc;
        total += align256(b);
    }
    *bytes = total;
    return WSX_OK;
}

int wsx_autotune_batch(const wsx_env_desc* const* descs, const wsx_policy* const* policies,
                       int32_t n, int32_t horizon, int32_t reps, void* workspace,
                       size_t workspace_bytes, wsx_tune_entry* best, void* stream) {
    size_t need = 0;
    int rc = wsx_autotune_batch_workspace_bytes(descs, n, horizon, &need);
    if (rc) return rc;
    if (!policies) return fail(WSX_EINVAL, "policies is NULL");
    if (reps < 1) return fail(WSX_EINVAL, "reps must be >= 1");
    if (!workspace || workspace_bytes < need)
        return fail(WSX_EINVAL, "workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    int kinds[2] = {0, 0}, n_kinds = 0;
    int64_t total_rows = 0;
    for (int i = 0; i < n; ++i) {
        KindInfo k;
        kind_info(descs[i]->kind, k);
        if (!policies[i] || policies[i]->dtype != k.dtype || policies[i]->h1 != k.hidden)
            return fail(WSX_EUNSUPPORTED, "no compiled kernel for policies[%d]", i);
        const int kd = descs[i]->kind;
        if (!(n_kinds > 0 && kinds[0] == kd) && !(n_kinds > 1 && kinds[1] == kd)) {
            if (n_kinds == 2) return fail(WSX_EUNSUPPORTED, "a batch mixes at most two kinds");
            kinds[n_kinds++] = kd;
        }
        total_rows += rows_of(descs[i]);
    }
    KindInfo k0;
    kind_info(kinds[0], k0);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "wsx_autotune_batch");

    // per set: its state block and trajectory inside the workspace
    std::vector<char*> base(n);
    std::vector<wsx_traj> trs(n);
    char* at = static_cast<char*>(workspace);
    for (int i = 0; i < n; ++i) {
        KindInfo k;
        kind_info(descs[i]->kind, k);
        const Trial T = trial_layout(k, descs[i]->kind, descs[i]->n_envs, rows_of(descs[i]), horizon);
        base[i] = at;
        wsx_traj& tr = trs[i];
        tr = wsx_traj{};
        tr.capacity = horizon;
        tr.obs = reinterpret_cast<float*>(at + T.off[0]);
        tr.action = at + T.off[1];
        tr.reward = reinterpret_cast<float*>(at + T.off[2]);
        tr.done = reinterpret_cast<uint8_t*>(at + T.off[3]);
        tr.value = reinterpret_cast<float*>(at + T.off[4]);
        tr.logp = reinterpret_cast<float*>(at + T.off[5]);
        tr.last_value = reinterpret_cast<float*>(at + T.off[6]);
        at += align256(T.total);
    }

    // candidate shapes: the fused kernels that run this mix, at full row
    // capacity and at the tile heights that spread all rows evenly over the CUs
    struct Cand {
        int tile_rows, waves, occupancy;
    };
    std::vector<Cand> cands;
    for (int i = 0; i < n_variants(); ++i) {
        const Variant& v = variant(i);
        const bool kinds_ok = n_kinds == 1 ? (v.kind == kinds[0] && v.kind2 == 0)
                                           : ((v.kind == kinds[0] && v.kind2 == kinds[1]) ||
                                              (v.kind == kinds[1] && v.kind2 == kinds[0]));
        if (!kinds_ok || v.dtype != k0.dtype || v.hidden != k0.hidden) continue;
        std::vector<int> heights = {v.tile_rows};
        if (kinds[0] != WSX_MARKET)
            for (int per = 1; per <= 8; ++per)
                heights.push_back((int)((total_rows + (int64_t)per * cus - 1) / ((int64_t)per * cus)));
        for (int t : heights) {
            Variant w;
            const bool runs_here =
                t >= 1 && t <= v.tile_rows &&
                (n_kinds == 1 ? find_variant(kinds[0], k0.dtype, k0.hidden, v.waves, t, v.occupancy, w)
                              : find_pair_variant(kinds[0], kinds[1], k0.dtype, k0.hidden, v.waves,
                                                  t, v.occupancy, w)) &&
                w.tile_rows == v.tile_rows;
            // every set must also have a single-kind kernel of this shape (env_create)
            for (int j = 0; runs_here && j < n_kinds; ++j) {
                Variant u;
                if (!find_variant(kinds[j], k0.dtype, k0.hidden, v.waves, t, v.occupancy, u) ||
                    u.waves != v.waves || u.occupancy != v.occupancy)
                    t = 0;
            }
            bool dup = false;
            for (const Cand& c : cands)
                dup = dup || (c.tile_rows == t && c.waves == v.waves && c.occupancy == v.occupancy);
            if (runs_here && t > 0 && !dup) cands.push_back({t, v.waves, v.occupancy});
        }
    }
    if (cands.empty()) return fail(WSX_EUNSUPPORTED, "no fused kernel runs this mix of kinds");

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e != hipSuccess) return hip_fail(e, "wsx_autotune_batch (events)");
    wsx_tune_entry win{};
    double win_ms = 0.0;
    std::vector<wsx_env*> envs(n, nullptr);
    std::vector<const wsx_traj*> tp(n);
    for (int i = 0; i < n; ++i) tp[i] = &trs[i];
    for (const Cand& c : cands) {
        for (int i = 0; i < n && !rc; ++i) {
            wsx_env_desc dd = *descs[i];
            dd.state = base[i];
            dd.tile_rows = c.tile_rows;
            dd.waves = c.waves;
            dd.occupancy = c.occupancy;
            rc = wsx_env_create(&dd, &envs[i]);
            if (!rc) rc = wsx_env_reset(envs[i], 0, stream);
        }
        if (!rc) rc = wsx_rollout_batch(envs.data(), policies, tp.data(), n, horizon, stream);
        std::vector<float> t;
        for (int r = 0; !rc && r < reps; ++r) {
            hipError_t he = hipEventRecord(ev0, s);
            if (he == hipSuccess &&
                (rc = wsx_rollout_batch(envs.data(), policies, tp.data(), n, horizon, stream)) == 0)
                he = hipEventRecord(ev1, s);
            if (he == hipSuccess && !rc) he = hipEventSynchronize(ev1);
            float m = 0.0f;
            if (he == hipSuccess && !rc) he = hipEventElapsedTime(&m, ev0, ev1);
            if (he != hipSuccess && !rc) rc = hip_fail(he, "wsx_autotune_batch (timing)");
            t.push_back(m);
        }
        for (int i = 0; i < n; ++i)
            if (envs[i]) {
                wsx_env_destroy(envs[i]);
                envs[i] = nullptr;
            }
        if (rc) break;
        std::sort(t.begin(), t.end());
        const double ms = t[t.size() / 2];
        if (win_ms == 0.0 || ms < win_ms) {
            win_ms = ms;
            win = {c.tile_rows, c.waves, c.occupancy, 0, 0.0};
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc) return rc;
    win.us_per_step = win_ms * 1000.0 / horizon;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int i = 0; i < n; ++i)
            put(g_table, Row{Key{descs[i]->kind, descs[i]->n_envs, rows_of(descs[i]), cus}, win});
    }
    if (best) *best = win;
    return WSX_OK;
}

int wsx_tune_lookup(int32_t kind, int64_t n_envs, int64_t n_rows, int32_t cus,
                    wsx_tune_entry* out) {
    if (!out) return fail(WSX_EINVAL, "out is NULL");
    if (!tune_lookup(kind, n_envs, n_rows, cus, *out))
        return fail(WSX_EINVAL, "no tuning entry for kind %d, %lld envs, %lld rows, %d CUs", kind,
                    (long long)n_envs, (long long)n_rows, cus);
    return WSX_OK;
}

int wsx_tune_save(const char* path) {
    if (!path) return fail(WSX_EINVAL, "path is NULL");
    std::vector<Row> rows;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        rows = g_table;
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(WSX_EINVAL, "cannot write %s", path);
    bool ok = std::fprintf(f, "# kind n_envs n_rows cus tile_rows waves occupancy chunk_steps "
                              "us_per_step\n") > 0;
    for (const Row& r : rows)
        ok = ok && std::fprintf(f, "%d %lld %lld %d %d %d %d %d %.6g\n", r.key.kind,
                                (long long)r.key.n_envs, (long long)r.key.n_rows, r.key.cus,
                                r.e.tile_rows, r.e.waves, r.e.occupancy, r.e.chunk_steps,
                                r.e.us_per_step) > 0;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? WSX_OK : fail(WSX_EINVAL, "writing %s failed", path);
}

int wsx_tune_load(const char* path) {
    if (!path) return fail(WSX_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(WSX_EINVAL, "cannot read %s", path);
    std::vector<Row> rows;
    char line[512];
    int lineno = 0;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        const char* p = line;
        while (*p == ' ' || *p == '\t') ++p;
        if (*p == '#' || *p == '\n' || *p == '\r' || *p == 0) continue;
        Row r{};
        long long ne = 0, nr = 0;
        char tail = 0;
        const int n = std::sscanf(p, "%d %lld %lld %d %d %d %d %d %lf %c", &r.key.kind, &ne, &nr,
                                  &r.key.cus, &r.e.tile_rows, &r.e.waves, &r.e.occupancy,
                                  &r.e.chunk_steps, &r.e.us_per_step, &tail);
        r.key.n_envs = ne;
        r.key.n_rows = nr;
        KindInfo k;
        Variant v;
        const bool ok = n == 9 && kind_info(r.key.kind, k) && ne > 0 && nr >= ne &&
                        r.key.cus > 0 && r.e.chunk_steps >= 0 && r.e.tile_rows > 0 &&
                        find_variant(r.key.kind, k.dtype, k.hidden, r.e.waves, r.e.tile_rows,
                                     r.e.occupancy, v) &&
                        v.waves == r.e.waves && v.occupancy == r.e.occupancy;
        if (!ok) {
            std::fclose(f);
            return fail(WSX_EINVAL, "%s:%d: not a tuning entry for a compiled kernel", path, lineno);
        }
        put(rows, r);
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Row& r : rows) put(g_table, r);
    return WSX_OK;
}

}  // extern "C"
