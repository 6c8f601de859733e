"""Environment sources for the user-kind composer tests: copies of two
built-in kinds (so their roll-outs must equal the built-in ones bit for bit)
and a new environment checked against a numpy re-implementation."""

# the built-in Pendulum, as user code
PENDULUM = r"""
struct UserEnv {
    static constexpr int KIND = WSX_USER_KIND, SD = 2, SR = 4, OD = 3, NACT = 0, LANES = 1;
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
        const float acc = 15.0f * s[2] + 3.0f * u;
        const float w = fminf(fmaxf(thd + acc * 0.05f, -8.0f), 8.0f);
        s[0] = th + w * 0.05f;
        s[1] = w;
        complete(s);
        done = false;
    }
};
"""

# the built-in CartPole, as user code
CARTPOLE = r"""
struct UserEnv {
    static constexpr int KIND = WSX_USER_KIND, SD = 4, SR = 4, OD = 4, NACT = 2, LANES = 1;
    __device__ static void complete(float*) {}
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
        const Words w = draw(key, t, row, PURPOSE_RESET, 0);
        for (int i = 0; i < 4; ++i) s[i] = -0.05f + 0.1f * unit_uniform(w.w[i]);
    }
    __device__ static void observe(const float* s, float* o) {
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
        const float inv_total = 1.0f / m_total;
        const float push = (force + m_pole * half_len * thd * thd * sn) * inv_total;
        const float thdd = (gravity * sn - cs * push) *
                           __builtin_amdgcn_rcpf(half_len * (4.0f / 3.0f - m_pole * cs * cs * inv_total));
        const float xdd = push - m_pole * half_len * thdd * cs * inv_total;
        s[0] = x + dt * xd;
        s[1] = xd + dt * xdd;
        s[2] = th + dt * thd;
        s[3] = thd + dt * thdd;
        const float th_limit = 0.20943951023931953f;
        done = fabsf(s[0]) > 2.4f || fabsf(s[2]) > th_limit;
        reward = 1.0f;
    }
};
"""

# a new environment: a point mass on a line pushed by a clipped force,
# reward -x^2 - 0.01 u^2, episode ends when |x| > 2; reset uniform in [-1, 1]^2
POINT_MASS = r"""
struct UserEnv {
    static constexpr int KIND = WSX_USER_KIND, SD = 2, SR = 2, OD = 2, NACT = 0, LANES = 1;
    __device__ static void complete(float*) {}
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
        const Words w = draw(key, t, row, PURPOSE_RESET, 0);
        s[0] = -1.0f + 2.0f * unit_uniform(w.w[0]);
        s[1] = -1.0f + 2.0f * unit_uniform(w.w[1]);
    }
    __device__ static void observe(const float* s, float* o) { o[0] = s[0]; o[1] = s[1]; }
    template <int G>
    __device__ static void step(float* s, int, float f, uint32_t, uint32_t, const RngKey&,
                                const EnvCtx&, int, float& reward, bool& done) {
        const float u = fminf(fmaxf(f, -1.0f), 1.0f);
        const float v = s[1] + 0.1f * u;
        const float x = s[0] + 0.1f * v;
        reward = -(x * x) - 0.01f * u * u;
        s[0] = x;
        s[1] = v;
        done = fabsf(x) > 2.0f;
    }
};
"""


def point_mass_step(x, v, f):
    """numpy float32 re-implementation of POINT_MASS's step."""
    import numpy as np
    f32 = np.float32
    u = np.clip(f.astype(f32), f32(-1), f32(1))
    v2 = (v + f32(0.1) * u).astype(f32)
    x2 = (x + f32(0.1) * v2).astype(f32)
    r = (-(x2 * x2) - f32(0.01) * u * u).astype(f32)
    return x2, v2, r, np.abs(x2) > f32(2)


# a new environment whose rows use four lanes: every lane moves the whole
# state, the reward's sum of squares is split over the lanes and combined
# with the library's group reduction
GROUP_WALK = r"""
struct UserEnv {
    static constexpr int KIND = WSX_USER_KIND, SD = 4, SR = 4, OD = 4, NACT = 0, LANES = 4;
    __device__ static void complete(float*) {}
    __device__ static void reset(float* s, const RngKey& key, uint32_t t, uint32_t row,
                                 const EnvCtx&) {
        const Words w = draw(key, t, row, PURPOSE_RESET, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = -1.0f + 2.0f * unit_uniform(w.w[i]);
    }
    __device__ static void observe(const float* s, float* o) {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = s[i];
    }
    template <int G>
    __device__ static void step(float* s, int, float a, uint32_t, uint32_t, const RngKey&,
                                const EnvCtx&, int sub, float& reward, bool& done) {
        const float u = fminf(fmaxf(a, -1.0f), 1.0f);
        float part = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            s[i] = 0.9f * s[i] + 0.1f * u * (float)(i + 1);
            if (i % G == sub) part += s[i] * s[i];
        }
        reward = -group_sum<G>(part);
        done = false;
    }
};
"""


def group_walk_step(s, a):
    """numpy float32 re-implementation of GROUP_WALK's step: s [n, 4], a [n]."""
    import numpy as np
    f32 = np.float32
    u = np.clip(a.astype(f32), f32(-1), f32(1))
    s2 = (f32(0.9) * s.astype(f32) + (f32(0.1) * u)[:, None] * np.arange(1, 5, dtype=f32)).astype(f32)
    return s2, -(s2 * s2).sum(axis=1)
