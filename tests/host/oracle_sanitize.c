/* The FP64 oracle (oracle/oracle.c, included as one translation unit) driven
 * through every entry point on small inputs of every kind, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_host_sanitizers.py: out-of-bounds accesses, leaks, signed
 * overflow and other undefined behaviour stop the run. Test infrastructure
 * only; the values are checked elsewhere (tests/test_oracle_*.py).        */
#include "../../oracle/oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;
static double unif(void)   /* [0, 1) */
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}
static double* randn(size_t n, double sd)
{
    double* a = (double*)malloc(sizeof(double) * n);
    for (size_t i = 0; i < n; ++i) a[i] = sd * (2.0 * unif() - 1.0) * 1.7;
    return a;
}

typedef struct {
    orc_mlp m;
    double *W1, *b1, *W2, *b2, *W3, *b3;
} policy;

static policy make_policy(int dtype, int d_in, int h, int n_head)
{
    policy p;
    p.W1 = randn((size_t)h * d_in, 0.1);
    p.b1 = randn(h, 0.1);
    p.W2 = randn((size_t)h * h, 0.1);
    p.b2 = randn(h, 0.1);
    p.W3 = randn((size_t)n_head * h, 0.1);
    p.b3 = randn(n_head, 0.1);
    /* quantise the weights to the format, as the real policies are */
    double* all[3] = {p.W1, p.W2, p.W3};
    size_t cnt[3] = {(size_t)h * d_in, (size_t)h * h, (size_t)n_head * h};
    for (int l = 0; l < 3; ++l)
        for (size_t i = 0; i < cnt[l]; ++i)
            all[l][i] = dtype == ORC_BF16 ? orc_round_bf16(all[l][i])
                        : dtype == ORC_FP8 ? ldexp(orc_round_fp8e4m3(ldexp(all[l][i], 10)), -10)
                                           : all[l][i];
    p.m.dtype = dtype;
    p.m.d_in = d_in;
    p.m.h1 = h;
    p.m.h2 = h;
    p.m.n_head = n_head;
    p.m.W1 = p.W1; p.m.b1 = p.b1; p.m.W2 = p.W2; p.m.b2 = p.b2; p.m.W3 = p.W3; p.m.b3 = p.b3;
    p.m.act_scale[0] = dtype == ORC_FP8 ? 1.0 / 16 : 1.0;
    p.m.act_scale[1] = dtype == ORC_FP8 ? 1.0 / 256 : 1.0;
    p.m.act_scale[2] = dtype == ORC_FP8 ? 1.0 / 256 : 1.0;
    return p;
}

static void free_policy(policy* p)
{
    free(p->W1); free(p->b1); free(p->W2); free(p->b2); free(p->W3); free(p->b3);
}

static void run_kind(int kind, int n_envs, int T, int dtype, int h)
{
    const int sd = orc_state_dim(kind), od = orc_obs_dim(kind), na = orc_n_actions(kind);
    int32_t* off = NULL;
    double* params = NULL;
    if (kind == ORC_MARKET) {
        off = (int32_t*)malloc(sizeof(int32_t) * (n_envs + 1));
        off[0] = 0;
        for (int e = 0; e < n_envs; ++e) off[e + 1] = off[e] + 1 + (int)(unif() * 9);
    }
    if (kind == ORC_REACTION) {
        params = (double*)malloc(sizeof(double) * (20 * 20 + 64 * 20 + 64 + 64));
        for (int i = 0; i < 20 * 20; ++i) params[i] = (i % 21 == 0) ? 1.0 : 0.0;
        for (int i = 0; i < 64 * 20; ++i) params[400 + i] = 6.0 * unif() - 3.0;
        for (int i = 0; i < 64; ++i) params[400 + 1280 + i] = 0.3 + 0.7 * unif();
        for (int i = 0; i < 64; ++i) params[400 + 1280 + 64 + i] = 2.0 * unif() - 1.0;
    }
    orc_env env = {kind, n_envs, off, params};
    const int64_t rows = orc_n_rows(&env);
    policy p = make_policy(dtype, od, h, (na ? na : 1) + 1);
    double log_std = -0.5;
    double* st = (double*)malloc(sizeof(double) * rows * sd);
    orc_env_reset(&env, 3, 1, 0, st);
    size_t n = (size_t)T * rows;
    orc_traj tr;
    tr.obs = (double*)malloc(sizeof(double) * n * od);
    tr.action = (double*)malloc(sizeof(double) * n);
    tr.reward = (double*)malloc(sizeof(double) * n);
    tr.done = (uint8_t*)malloc(n);
    tr.value = (double*)malloc(sizeof(double) * n);
    tr.logp = (double*)malloc(sizeof(double) * n);
    tr.last_value = (double*)malloc(sizeof(double) * rows);
    tr.margin_action = (double*)malloc(sizeof(double) * n);
    tr.margin_done = (double*)malloc(sizeof(double) * n);
    if (orc_rollout(&env, &p.m, &log_std, 3, 1, 0, T, st, &tr) != 0) {
        fprintf(stderr, "rollout rejected kind %d\n", kind);
        exit(1);
    }
    double* ret = (double*)malloc(sizeof(double) * n);
    double* adv = (double*)malloc(sizeof(double) * n);
    orc_returns_gae(T, rows, tr.reward, tr.value, tr.done, tr.last_value, 0.99, 0.95, 1, ret, adv);
    if (T <= 8) orc_gae_bruteforce(T, rows, tr.reward, tr.value, tr.done, tr.last_value, 0.99,
                                   0.95, 0, ret, adv);
    /* adoption with the oracle's own codes (random codes also exercise the
     * flip paths) */
    double* c1 = randn((size_t)rows * h, 0.5);
    double* c2 = randn((size_t)rows * h, 0.5);
    double* head = (double*)malloc(sizeof(double) * rows * p.m.n_head);
    double* hb = (double*)malloc(sizeof(double) * rows * p.m.n_head);
    int32_t* flips = (int32_t*)malloc(sizeof(int32_t) * rows * 2);
    double* ratio = (double*)malloc(sizeof(double) * rows * 2);
    orc_mlp_adopt(&p.m, rows, tr.obs, c1, c2, head, hb, flips, ratio);
    uint32_t* rid = (uint32_t*)malloc(sizeof(uint32_t) * rows);
    for (int64_t r = 0; r < rows; ++r) rid[r] = (uint32_t)r;
    double* a = (double*)malloc(sizeof(double) * rows);
    double* lp = (double*)malloc(sizeof(double) * rows);
    double* mg = (double*)malloc(sizeof(double) * rows);
    orc_sample_rows(rows, p.m.n_head, na, head, &log_std, 3, 5, rid, 1, a, lp, mg);
    /* the actor-critic gradient and Adam (FP32 and BF16 policies) */
    if (dtype != ORC_FP8) {
        double* g[7];
        size_t sz[7] = {(size_t)h * od, (size_t)h, (size_t)h * h, (size_t)h,
                        (size_t)p.m.n_head * h, (size_t)p.m.n_head, 1};
        for (int i = 0; i < 7; ++i) g[i] = (double*)calloc(sz[i], sizeof(double));
        if (orc_ac_grad(&p.m, na, &log_std, (int64_t)n, tr.obs, tr.action, adv, ret, 0.5, 0.01,
                        dtype == ORC_BF16, g[0], g[1], g[2], g[3], g[4], g[5], g[6]) != 0) {
            fprintf(stderr, "ac_grad rejected kind %d\n", kind);
            exit(1);
        }
        double* th = randn(sz[2], 0.1);
        double* m = (double*)calloc(sz[2], sizeof(double));
        double* v = (double*)calloc(sz[2], sizeof(double));
        for (int t = 1; t <= 3; ++t) orc_adam((int64_t)sz[2], th, g[2], m, v, t, 1e-3, 0.9, 0.999, 1e-8);
        free(th); free(m); free(v);
        for (int i = 0; i < 7; ++i) free(g[i]);
    }
    if (kind == ORC_CARTPOLE) {
        double* s0 = (double*)malloc(sizeof(double) * rows * 4);
        orc_env_reset(&env, 3, 1, 0, s0);
        double* o32 = (double*)malloc(sizeof(double) * n * 4);
        double* a32 = (double*)malloc(sizeof(double) * n);
        orc_cartpole_rollout_f32(&p.m, rows, 3, 1, 0, T, s0, o32, a32);
        free(s0); free(o32); free(a32);
    }
    free(rid); free(a); free(lp); free(mg);
    free(c1); free(c2); free(head); free(hb); free(flips); free(ratio);
    free(ret); free(adv);
    free(tr.obs); free(tr.action); free(tr.reward); free(tr.done); free(tr.value);
    free(tr.logp); free(tr.last_value); free(tr.margin_action); free(tr.margin_done);
    free(st);
    free_policy(&p);
    free(off);
    free(params);
}

int main(void)
{
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    run_kind(ORC_CARTPOLE, 17, 30, ORC_F32, 64);
    run_kind(ORC_PENDULUM, 13, 8, ORC_BF16, 32);
    run_kind(ORC_ACROBOT, 11, 12, ORC_BF16, 32);
    run_kind(ORC_MARKET, 5, 6, ORC_BF16, 32);
    run_kind(ORC_REACTION, 6, 7, ORC_FP8, 64);
    printf("oracle under sanitizers: ok\n");
    return 0;
}
