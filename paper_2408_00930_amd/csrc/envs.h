// envs.h -- FP32 environment dynamics on the device.
//
// The example families of arXiv 2408.00930, App. C (classic control, a
// multi-agent economy, a noisy potential-energy walk). The paper gives no
// equations; these follow the project's specification: Lagrangian mechanics
// for the classic-control bodies, the market and reaction rules read from the
// workload descriptions. Every function works on one row (agent) held in
// registers; the market's cross-agent sums are done by the kernels. The
// register state has SR >= SD entries: the SD stored ones, then values derived
// from them (the sine and cosine of the angles, which observe() and the next
// step use), filled by complete() after a load and kept current by reset()
// and step().
#pragma once

#include "device.h"

namespace wsx {

struct EnvCtx {
    const float* lds_params;  // reaction: potential block staged in LDS
    double* cache;            // reaction: this row's FP64 energy terms, entry j at
    int cache_stride;         //   cache[j * cache_stride]
};

// ------------------------------------------------------------ CartPole --
// Cart (mass 1) with a hinged uniform pole (mass 0.1, half-length 0.5), force
// +-10, explicit Euler dt 0.02; ends when |x| > 2.4 or |theta| > 12 degrees.
struct CartPole {
    static constexpr int KIND = 1, SD = 4, SR = 4, OD = 4, NACT = 2, LANES = 1;
    __device__ static void complete(float*) {}
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
        const Words w = draw(key, t, row, PURPOSE_RESET, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = -0.05f + 0.1f * unit_uniform(w.w[i]);
    }
    __device__ static void observe(const float* s, float* o) {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = s[i];
    }
    template <int G>
    __device__ static void step(float* s, int action, float, uint32_t, uint32_t, const RngKey&,
                                const EnvCtx&, int, float& reward, bool& done) {
        const float gravity = 9.8f, m_pole = 0.1f, m_total = 1.1f, half_len = 0.5f;
        const float dt = 0.02f;
        const float force = action == 1 ? 10.0f : -10.0f;
        const float x = s[0], xd = s[1], th = s[2], thd = s[3];
        float sn, cs;
        sin_cos(th, sn, cs);
        // divisions as products with reciprocals (the constant one folded,
        // the other v_rcp_f32): the per-row phase is a latency chain, and an
        // IEEE division is ten dependent instructions
        const float inv_total = 1.0f / m_total;
        const float push = (force + m_pole * half_len * thd * thd * sn) * inv_total;
        const float thdd = (gravity * sn - cs * push) *
                           __builtin_amdgcn_rcpf(half_len * (4.0f / 3.0f - m_pole * cs * cs * inv_total));
        const float xdd = push - m_pole * half_len * thdd * cs * inv_total;
        s[0] = x + dt * xd;
        s[1] = xd + dt * xdd;
        s[2] = th + dt * thd;
        s[3] = thd + dt * thdd;
        const float th_limit = 0.20943951023931953f;  // 12 degrees
        done = fabsf(s[0]) > 2.4f || fabsf(s[2]) > th_limit;
        reward = 1.0f;
    }
};

__device__ __forceinline__ float wrap_pi(float a) {
    // a - 2 pi floor((a + pi) / (2 pi)), in [-pi, pi)
    const float two_pi = 6.283185307179586f;
    return a - two_pi * floorf((a + 3.141592653589793f) * 0.15915494309189535f);
}

// ------------------------------------------------------------ Pendulum --
// Rod (m 1, l 1) under gravity 10 about its end, theta 0 upright, torque
// clipped to 2; semi-implicit Euler dt 0.05, rate clipped to 8.
struct Pendulum {
    // register state: theta, theta', sin theta, cos theta
    static constexpr int KIND = 2, SD = 2, SR = 4, OD = 3, NACT = 0, LANES = 1;
    __device__ static void complete(float* s) { sin_cos(s[0], s[2], s[3]); }
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
        const Words w = draw(key, t, row, PURPOSE_RESET, 0);
        s[0] = -3.141592653589793f + 6.283185307179586f * unit_uniform(w.w[0]);
        s[1] = -1.0f + 2.0f * unit_uniform(w.w[1]);
        complete(s);
    }
    __device__ static void observe(const float* s, float* o) {
        o[0] = s[3];
        o[1] = s[2];
        o[2] = s[1];
    }
    template <int G>
    __device__ static void step(float* s, int, float torque, uint32_t, uint32_t, const RngKey&,
                                const EnvCtx&, int, float& reward, bool& done) {
        const float u = fminf(fmaxf(torque, -2.0f), 2.0f);
        const float th = s[0], thd = s[1];
        const float a = wrap_pi(th);
        reward = -(a * a + 0.1f * thd * thd + 0.001f * u * u);
        // theta'' = 3 g / (2 l) sin(theta) + 3 u / (m l^2)
        const float acc = 15.0f * s[2] + 3.0f * u;
        const float w = fminf(fmaxf(thd + acc * 0.05f, -8.0f), 8.0f);
        s[0] = th + w * 0.05f;
        s[1] = w;
        complete(s);
        done = false;
    }
};

// ------------------------------------------------------------- Acrobot --
// Two links (length 1, centre of mass 0.5, mass 1, inertia 1), elbow torque
// in [-1, 1], RK4 over dt 0.2; ends when the tip is more than one link length
// above the base.
struct Acrobot {
    // register state: theta1, theta2, rates, then sin / cos of both angles
    static constexpr int KIND = 3, SD = 4, SR = 8, OD = 6, NACT = 0, LANES = 1;
    __device__ static void complete(float* s) {
        sin_cos(s[0], s[4], s[5]);
        sin_cos(s[1], s[6], s[7]);
    }
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
        const Words w = draw(key, t, row, PURPOSE_RESET, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = -0.1f + 0.2f * unit_uniform(w.w[i]);
        complete(s);
    }
    __device__ static void observe(const float* s, float* o) {
        o[0] = s[5];
        o[1] = s[4];
        o[2] = s[7];
        o[3] = s[6];
        o[4] = s[2];
        o[5] = s[3];
    }
    // Manipulator equations M(q) q'' + C(q, q') + G(q) = (0, tau) solved for
    // q'' with the 2x2 inertia matrix of the two links (Cramer's rule);
    // sin(q1 + q2) by the angle-addition formula. s1..c2: sin / cos of q1, q2.
    __device__ static void deriv(const float* q, float tau, float s1, float c1, float s2, float c2,
                                 float* dq) {
        const float g = 9.8f;
        const float m11 = 0.25f + (1.0f + 0.25f + c2) + 2.0f;  // lc1^2 + (l1^2+lc2^2+2 l1 lc2 c2) + I1 + I2
        const float m12 = (0.25f + 0.5f * c2) + 1.0f;
        const float m22 = 0.25f + 1.0f;
        const float w1 = q[2], w2 = q[3];
        const float cor1 = -0.5f * s2 * (w2 * w2 + 2.0f * w1 * w2);
        const float cor2 = 0.5f * s2 * w1 * w1;
        const float grav2 = 0.5f * g * __builtin_fmaf(s1, c2, c1 * s2);
        const float grav1 = 1.5f * g * s1 + grav2;
        const float rhs1 = -(cor1 + grav1);
        const float rhs2 = tau - cor2 - grav2;
        const float inv_det = __builtin_amdgcn_rcpf(m11 * m22 - m12 * m12);   // det >= 2.56
        dq[0] = w1;
        dq[1] = w2;
        dq[2] = (m22 * rhs1 - m12 * rhs2) * inv_det;
        dq[3] = (m11 * rhs2 - m12 * rhs1) * inv_det;
    }
    template <int G>
    __device__ static void step(float* s, int, float torque, uint32_t, uint32_t, const RngKey&,
                                const EnvCtx&, int, float& reward, bool& done) {
        const float tau = fminf(fmaxf(torque, -1.0f), 1.0f);
        const float h = 0.2f;
        float k1[4], k2[4], k3[4], k4[4], y[4];
        // sin / cos of a stage's angles (|angle| below about 10: the wrapped
        // angle plus h times a stage rate of up to ~9 pi) from the hardware
        // instructions, whose error there (below about 8e-7) moves the step's
        // result by ~1e-6 of its scale; the state's own sin / cos (the
        // observation) stay exact to about an ulp (complete)
        float a1, b1, a2, b2;
        deriv(s, tau, s[4], s[5], s[6], s[7], k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = s[i] + 0.5f * h * k1[i];
        sin_cos_hw(y[0], a1, b1);
        sin_cos_hw(y[1], a2, b2);
        deriv(y, tau, a1, b1, a2, b2, k2);
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = s[i] + 0.5f * h * k2[i];
        sin_cos_hw(y[0], a1, b1);
        sin_cos_hw(y[1], a2, b2);
        deriv(y, tau, a1, b1, a2, b2, k3);
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = s[i] + h * k3[i];
        sin_cos_hw(y[0], a1, b1);
        sin_cos_hw(y[1], a2, b2);
        deriv(y, tau, a1, b1, a2, b2, k4);
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = s[i] + (h / 6.0f) * (k1[i] + 2.0f * k2[i] + 2.0f * k3[i] + k4[i]);
        s[0] = wrap_pi(y[0]);
        s[1] = wrap_pi(y[1]);
        s[2] = fminf(fmaxf(y[2], -12.566370614359172f), 12.566370614359172f);
        s[3] = fminf(fmaxf(y[3], -28.274333882308138f), 28.274333882308138f);
        complete(s);
        const float s1 = s[4], c1 = s[5], s2 = s[6], c2 = s[7];
        const float tip = -c1 - __builtin_fmaf(c1, c2, -s1 * s2);   // -cos q1 - cos(q1 + q2)
        done = tip > 1.0f;
        reward = done ? 0.0f : -1.0f;
    }
};

// -------------------------------------------------------------- Market --
// Per agent: 32-d state; the env-wide demand and supply sums are formed by
// the kernels (exactly, in integer units) between decide() and settle().
// LANES: how many lanes of a group can share a row's sampling and dynamics.
struct Market {
    static constexpr int KIND = 4, SD = 32, SR = 32, OD = 32, NACT = 50, LANES = 4;
    __device__ static void complete(float*) {}
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
#pragma unroll
        for (int sub = 0; sub < 8; ++sub) {
            const Words w = draw(key, t, row, PURPOSE_RESET, (uint32_t)sub);
            gauss_pair(unit_uniform(w.w[0]), unit_uniform(w.w[1]), s[4 * sub], s[4 * sub + 1]);
            gauss_pair(unit_uniform(w.w[2]), unit_uniform(w.w[3]), s[4 * sub + 2], s[4 * sub + 3]);
        }
    }
    __device__ static void observe(const float* s, float* o) {
#pragma unroll
        for (int i = 0; i < 32; ++i) o[i] = s[i];
    }
    // Action a -> labour level k in 0..9 (labour k/9) and trade level j in
    // 0..4 (trade (j-2)/2). Demand in half units: max(j-2, 0). Supply in
    // 1/18 units: 2k + 9 max(2-j, 0).
    __device__ static void decide(int a, int& demand_half, int& supply_18th) {
        const int k = a % 10, j = a / 10;
        demand_half = j > 2 ? j - 2 : 0;
        supply_18th = 2 * k + 9 * (j < 2 ? 2 - j : 0);
    }
    // The terms of a settled step: labour, trade, consumption, reward and the
    // log price, from the action and the env-wide integer sums. Reciprocals
    // stand in for the four divisions (k / 9, S / 18, the price ratio and
    // bought / price), each within an ulp or two, and the hardware log for
    // logf / log1pf (a few 1e-7 absolute): this is a per-row dependent chain
    // and a full-precision division or log is ten to fifteen instructions.
    __device__ static void terms(int a, int demand_half_sum, int supply_18th_sum, float& labour,
                                 float& trade, float& cons, float& reward, float& lp) {
        const int k = a % 10, j = a / 10;
        labour = (float)k * (1.0f / 9.0f);
        trade = (float)(j - 2) * 0.5f;
        const float eps = 1e-3f;
        const float demand = (float)demand_half_sum * 0.5f;
        const float supply = (float)supply_18th_sum * (1.0f / 18.0f);
        const float num = demand + eps, den = supply + eps;
        const float price = num * __builtin_amdgcn_rcpf(den);
        const float sold = trade < 0.0f ? -trade : 0.0f;
        const float bought = trade > 0.0f ? trade : 0.0f;
        cons = fmaxf(0.0f, labour - sold + bought * (den * __builtin_amdgcn_rcpf(num)));
        reward = log_hw(1.0f + cons) - 0.1f * labour * labour;
        lp = log_hw(price);
    }
    __device__ static void settle(float* s, int a, int demand_half_sum, int supply_18th_sum,
                                  float& reward) {
        float labour, trade, cons, lp;
        terms(a, demand_half_sum, supply_18th_sum, labour, trade, cons, reward, lp);
        s[0] = 0.9f * s[0] + 0.1f * (cons - 0.5f);
        s[1] = lp;
        s[2] = labour;
        s[3] = trade;
        s[4] = cons;
#pragma unroll
        for (int i = 5; i < 32; ++i) s[i] = 0.99f * s[i];
    }
    // The same update on a slice: the lanes of a row's group of G hold the
    // state entries i = sub + j G (j < 32 / G), each updated as above.
    template <int G>
    __device__ static void settle_slice(float (&s)[32 / G], int sub, int a, int demand_half_sum,
                                        int supply_18th_sum, float& reward) {
        float labour, trade, cons, lp;
        terms(a, demand_half_sum, supply_18th_sum, labour, trade, cons, reward, lp);
#pragma unroll
        for (int q = 0; q < 32 / G; ++q) {
            const int i = sub + q * G;
            const float v = s[q];
            s[q] = i == 0   ? 0.9f * v + 0.1f * (cons - 0.5f)
                   : i == 1 ? lp
                   : i == 2 ? labour
                   : i == 3 ? trade
                   : i == 4 ? cons
                            : 0.99f * v;
        }
    }
};

// ------------------------------------------------------------ Reaction --
// 20-D walk on E(x) = x^T A x / 2 + sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2))
// plus 0.05 N(0,1) noise per evaluation. The LDS parameter block is A (400),
// centres (64 x 20), widths (64; staged in LDS as -log2(e)/(2 w^2)), amplitudes (64).
struct Reaction {
    static constexpr int KIND = 5, SD = 21, SR = 21, OD = 20, NACT = 40, NDIM = 20, NG = 64, LANES = 16;
    __device__ static void complete(float*) {}
    static constexpr int PARAM_FLOATS = NDIM * NDIM + NG * NDIM + NG + NG;
    // Per row, the energy's terms in FP64 (the row's cache): y = A x (NDIM
    // entries), then d_k = |x - c_k|^2 (NG entries). A move of coordinate c by
    // dl (the exact difference of the FP32 coordinates) updates them by
    // y_i += dl A_ic and d_k += dl (2 (x_c - c_kc) + dl), which are exact
    // identities: the cache stays the FP64 value of its definition (rounding
    // of order 1e-16 per step), and a step costs O(NDIM + NG) instead of
    // O(NDIM^2 + NG NDIM). Lane `sub` of the row's G lanes owns entries
    // i = sub + m G of y and k = sub + m G of d.
    static constexpr int NCACHE = NDIM + NG;
    template <int G>
    __device__ static void cache_init(const float* x, const float* p, const EnvCtx& c, int sub) {
        const float* A = p;
        const float* cen = p + NDIM * NDIM;
#pragma unroll
        for (int m = 0; m < (NDIM + G - 1) / G; ++m) {
            const int i = sub + m * G;
            if (i < NDIM) {
                double y = 0.0;
#pragma unroll
                for (int j = 0; j < NDIM; ++j) y = __builtin_fma((double)A[i * NDIM + j], (double)x[j], y);
                c.cache[i * c.cache_stride] = y;
            }
        }
#pragma unroll
        for (int m = 0; m < NG / G; ++m) {
            const int k = sub + m * G;
            double d2 = 0.0;
#pragma unroll
            for (int i = 0; i < NDIM; ++i) {
                const double d = (double)x[i] - (double)cen[k * NDIM + i];
                d2 = __builtin_fma(d, d, d2);
            }
            c.cache[(NDIM + k) * c.cache_stride] = d2;
        }
    }
    template <int G>
    __device__ static void cache_move(int coord, float x_old, float x_new, const float* p,
                                      const EnvCtx& c, int sub) {
        const float* A = p;
        const float* cen = p + NDIM * NDIM;
        const double dl = (double)x_new - (double)x_old;   // exact
#pragma unroll
        for (int m = 0; m < (NDIM + G - 1) / G; ++m) {
            const int i = sub + m * G;
            if (i < NDIM) {
                double& y = c.cache[i * c.cache_stride];
                y = __builtin_fma(dl, (double)A[i * NDIM + coord], y);
            }
        }
#pragma unroll
        for (int m = 0; m < NG / G; ++m) {
            const int k = sub + m * G;
            double& d2 = c.cache[(NDIM + k) * c.cache_stride];
            const double two_off = 2.0 * ((double)x_old - (double)cen[k * NDIM + coord]) + dl;
            d2 = __builtin_fma(dl, two_off, d2);
        }
    }
    // E(x) = x^T y / 2 + sum_k a_k exp(-d_k / (2 w_k^2)) from the cache, the
    // lane's terms in FP32, summed over the row's lanes; every lane returns
    // the same total.
    template <int G>
    __device__ static float energy(const float* x, const float* p, const EnvCtx& c, int sub) {
        float xs[(NDIM + G - 1) / G];
#pragma unroll
        for (int m = 0; m < (NDIM + G - 1) / G; ++m) {
            const int i = sub + m * G;
            float xi = 0.0f;
#pragma unroll
            for (int j = 0; j < NDIM; ++j) xi = j == i ? x[j] : xi;
            xs[m] = xi;
        }
        return energy_slice<G>(xs, p, c, sub);
    }
    // The same from the lane's own coordinates xs[m] = x[sub + m G]. Terms
    // past the last coordinate add zero (the running sum is never -0, so the
    // total is unchanged) instead of branching.
    template <int G>
    __device__ static float energy_slice(const float* xs, const float* p, const EnvCtx& c, int sub) {
        const float* nhw = p + NDIM * NDIM + NG * NDIM;
        const float* amp = nhw + NG;
        float part = 0.0f;
#pragma unroll
        for (int m = 0; m < (NDIM + G - 1) / G; ++m) {
            const int i = sub + m * G;
            const float t = 0.5f * xs[m] * (float)c.cache[(i < NDIM ? i : NDIM - 1) * c.cache_stride];
            part += i < NDIM ? t : 0.0f;
        }
#pragma unroll
        for (int m = 0; m < NG / G; ++m) {
            const int k = sub + m * G;
            part += amp[k] * __builtin_amdgcn_exp2f((float)c.cache[(NDIM + k) * c.cache_stride] * nhw[k]);
        }
        return group_sum<G>(part);
    }
    // The standard normal of the energy noise of the state reached at step t
    // (the cosine branch of the NOISE block (t, row)).
    __device__ static float noise_normal(const RngKey& key, uint32_t t, uint32_t row) {
        const Words w = draw(key, t, row, PURPOSE_NOISE, 0);
        float zc, zs;
        gauss_pair(unit_uniform(w.w[0]), unit_uniform(w.w[1]), zc, zs);
        return zc;
    }
    template <int G>
    __device__ static float noisy_energy(const float* x, const RngKey& key, uint32_t t, uint32_t row,
                                         const EnvCtx& c, int sub) {
        return energy<G>(x, c.lds_params, c, sub) + 0.05f * noise_normal(key, t, row);
    }
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx& c) {
#pragma unroll
        for (int sub = 0; sub < 5; ++sub) {
            const Words w = draw(key, t, row, PURPOSE_RESET, (uint32_t)sub);
#pragma unroll
            for (int i = 0; i < 4; ++i) s[4 * sub + i] = -3.0f + 6.0f * unit_uniform(w.w[i]);
        }
        cache_init<1>(s, c.lds_params, c, 0);
        s[20] = noisy_energy<1>(s, key, t, row, c, 0);
    }
    __device__ static void observe(const float* s, float* o) {
#pragma unroll
        for (int i = 0; i < 20; ++i) o[i] = s[i];
    }
    template <int G>
    __device__ static void step(float* s, int a, float, uint32_t t, uint32_t row, const RngKey& key,
                                const EnvCtx& c, int sub, float& reward, bool& done) {
        step_noise<G>(s, a, noise_normal(key, t + 1, row), c, sub, reward);
        done = false;
    }
    // What a lane's step reads that does not depend on the move: its cache
    // entries (y_i, i = sub + m G; d_k, k = sub + m G) and its Gaussians'
    // -log2(e)/(2 w^2) and amplitudes, loaded ahead so that the move waits only for
    // the two coordinate-dependent parameter reads.
    template <int G>
    struct Lane {
        static constexpr int NX = (NDIM + G - 1) / G, NK = NG / G;
        double y[NX], d[NK];
        float nhw[NK], amp[NK];
    };
    template <int G>
    __device__ static void lane_load(Lane<G>& l, const EnvCtx& c, int sub) {
        const float* nhw = c.lds_params + NDIM * NDIM + NG * NDIM;
        const float* amp = nhw + NG;
#pragma unroll
        for (int m = 0; m < Lane<G>::NX; ++m) {
            const int i = sub + m * G;
            l.y[m] = c.cache[(i < NDIM ? i : NDIM - 1) * c.cache_stride];
        }
#pragma unroll
        for (int m = 0; m < Lane<G>::NK; ++m) {
            const int k = sub + m * G;
            l.d[m] = c.cache[(NDIM + k) * c.cache_stride];
            l.nhw[m] = nhw[k];
            l.amp[m] = amp[k];
        }
    }
    // The step on a row whose G lanes each hold only their own coordinates
    // xs[m] = x[sub + m G] (and every lane the energy `en`): the moved
    // coordinate comes from the lane that holds it (`base` is the group's
    // first lane in the wave); the cache update and the energy are those of
    // cache_move and energy_slice, from the lane's preloaded entries.
    template <int G>
    __device__ static void step_slice(float* xs, float& en, Lane<G>& l, int a, float z,
                                      const EnvCtx& c, int sub, int base, float& reward) {
        constexpr int NX = Lane<G>::NX, NK = Lane<G>::NK;
        const float* A = c.lds_params;
        const float* cen = c.lds_params + NDIM * NDIM;
        const int coord = a >> 1;
        const float delta = (a & 1) ? -0.05f : 0.05f;
        const int owner = coord % G, jm = coord / G;
        float held = xs[0];
#pragma unroll
        for (int m = 1; m < NX; ++m) held = jm == m ? xs[m] : held;
        const float x_old = __shfl(held, base + owner);
        const float x_new = x_old + delta;
#pragma unroll
        for (int m = 0; m < NX; ++m) xs[m] = (sub == owner && jm == m) ? x_new : xs[m];
        const double dl = (double)x_new - (double)x_old;   // exact
#pragma unroll
        for (int m = 0; m < NX; ++m) {
            const int i = sub + m * G;
            if (i < NDIM) {
                l.y[m] = __builtin_fma(dl, (double)A[i * NDIM + coord], l.y[m]);
                c.cache[i * c.cache_stride] = l.y[m];
            }
        }
#pragma unroll
        for (int m = 0; m < NK; ++m) {
            const int k = sub + m * G;
            const double two_off = 2.0 * ((double)x_old - (double)cen[k * NDIM + coord]) + dl;
            l.d[m] = __builtin_fma(dl, two_off, l.d[m]);
            c.cache[(NDIM + k) * c.cache_stride] = l.d[m];
        }
        float part = 0.0f;
#pragma unroll
        for (int m = 0; m < NX; ++m) {
            const int i = sub + m * G;
            const float t = 0.5f * xs[m] * (float)l.y[m];
            part += i < NDIM ? t : 0.0f;
        }
#pragma unroll
        for (int m = 0; m < NK; ++m) part += l.amp[m] * __builtin_amdgcn_exp2f((float)l.d[m] * l.nhw[m]);
        const float e_new = group_sum<G>(part) + 0.05f * z;
        reward = -(e_new - en);
        en = e_new;
    }
    // The step with its noise normal z already drawn (noise_normal(key, t + 1,
    // row)); never terminates.
    template <int G>
    __device__ static void step_noise(float* s, int a, float z, const EnvCtx& c, int sub,
                                      float& reward) {
        const int coord = a >> 1;
        const float delta = (a & 1) ? -0.05f : 0.05f;
        // a select per coordinate keeps the state in registers (a branch on
        // the coordinate would index the array dynamically)
        float x_old = 0.0f, x_new = 0.0f;
#pragma unroll
        for (int i = 0; i < 20; ++i) {
            const float moved = s[i] + delta;
            x_old = i == coord ? s[i] : x_old;
            x_new = i == coord ? moved : x_new;
            s[i] = i == coord ? moved : s[i];
        }
        cache_move<G>(coord, x_old, x_new, c.lds_params, c, sub);
        const float e_new = energy<G>(s, c.lds_params, c, sub) + 0.05f * z;
        reward = -(e_new - s[20]);
        s[20] = e_new;
    }
};

}  // namespace wsx
