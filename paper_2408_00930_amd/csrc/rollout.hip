// rollout.hip -- the roll-out kernels of the built-in environment kinds
// (arXiv 2408.00930, Sec. 2 and App. B): the fused form's templates
// (rollout_kernels.h) instantiated for each compiled shape, the plain form
// (per step a policy kernel, a sample kernel and a step kernel with HBM round
// trips for the intermediates: the comparison baseline) and the dispatch.
#include "rollout_kernels.h"

namespace wsx {
// ---------------------------------------------------------- plain form --
template <class E>
__global__ void k_plain_observe(EnvArgs env, TrajArgs tr, int horizon) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= env.n_rows) return;
    float s[E::SR];
    load_state<E>(env, row, s);
    float o[E::OD];
    E::observe(s, o);
#pragma unroll
    for (int k = 0; k < E::OD; ++k) {
        env.obs_scratch[row * E::OD + k] = o[k];
        if (horizon > 0) tr.obs[row * E::OD + k] = o[k];
    }
}

// Policy over one tile of rows per workgroup: obs_scratch -> head_scratch.
// TRACE also writes the quantised hidden-layer outputs ([rows][H] codes of the
// policy format) to act1 / act2; the arithmetic is the fused kernel's.
template <class E, int DT, int H, int NW, int NT, int HS, int OCC, bool TRACE>
__device__ __forceinline__ void policy_tile(const EnvArgs& env, const PolicyArgs& pol, char* act1,
                                            char* act2) {
    using HO = HeadOf<E>;
    using L = Mlp<DT, H, NW, NT, kin_of<E, DT>(), HO::NHP, HS, OCC, TRACE>;
    constexpr int R = L::R;
    __shared__ __attribute__((aligned(16))) char smem[L::BYTES];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    L mlp;
    mlp.load(pol, smem, wave, lane, tid);
    const float inv_q0 = DT == DT_FP8 ? 1.0f / pol.act_scale[0] : 1.0f;
    for (int i = tid; i < R * L::P_IN / 4; i += NW * 64)
        reinterpret_cast<uint32_t*>(smem + L::OFF_IN)[i] = 0u;
    __syncthreads();
    const Tile tl = tile_of(env, blockIdx.x);
    if constexpr (TRACE) {
        mlp.tr_act[0] = act1 + (size_t)tl.row0 * H * L::EB;
        mlp.tr_act[1] = act2 + (size_t)tl.row0 * H * L::EB;
        mlp.tr_rows = tl.row1 - tl.row0;
    }
    const bool valid = tid < R && tl.row0 + tid < tl.row1;
    const int row = valid ? tile_row(env, tl.row0 + tid) : 0;
    if (valid) {
        float o[E::OD];
#pragma unroll
        for (int k = 0; k < E::OD; ++k) o[k] = env.obs_scratch[(size_t)row * E::OD + k];
        L::template put_obs<E::OD, 1>(smem, tid, o, inv_q0, 0);
    }
    __syncthreads();
    mlp.forward(smem, wave, lane);
    __syncthreads();
    if (valid) {
        float b3[HO::NH];
#pragma unroll
        for (int j = 0; j < HO::NH; ++j) b3[j] = pol.b3[j];
        float h[HO::NH];
        L::template head_row<HO::NH>(smem, b3, tid, h);
#pragma unroll
        for (int j = 0; j < HO::NH; ++j) env.head_scratch[(size_t)row * HO::NH + j] = h[j];
    }
}

template <class E, int DT, int H, int NW, int NT, int HS, int OCC>
__global__ void __attribute__((amdgpu_flat_work_group_size(NW * 64, NW * 64),
                               amdgpu_waves_per_eu(OCC)))
k_plain_policy(EnvArgs env, PolicyArgs pol) {
    policy_tile<E, DT, H, NW, NT, HS, OCC, false>(env, pol, nullptr, nullptr);
}

template <class E, int DT, int H, int NW, int NT, int HS, int OCC>
__global__ void __attribute__((amdgpu_flat_work_group_size(NW * 64, NW * 64),
                               amdgpu_waves_per_eu(OCC)))
k_policy_trace(EnvArgs env, PolicyArgs pol, char* act1, char* act2) {
    policy_tile<E, DT, H, NW, NT, HS, OCC, true>(env, pol, act1, act2);
}

template <class E, int H>
__global__ void __launch_bounds__(64) k_plain_policy_rw(EnvArgs env, PolicyArgs pol) {
    policy_row_rw<E, H, false>(env, pol, nullptr, nullptr);
}

template <class E, int H>
__global__ void __launch_bounds__(64) k_policy_trace_rw(EnvArgs env, PolicyArgs pol, char* act1,
                                                        char* act2) {
    policy_row_rw<E, H, true>(env, pol, reinterpret_cast<float*>(act1),
                              reinterpret_cast<float*>(act2));
}

// Plain sampling: G lanes per row, the same group code as the fused kernel.
template <class E, int G>
__global__ void __launch_bounds__(256) k_plain_sample(EnvArgs env, PolicyArgs pol, TrajArgs tr,
                                                      int step) {
    using HO = HeadOf<E>;
    using B = Block<E, G>;
    constexpr int C = B::C;
    const int sub = threadIdx.x % G;
    const int64_t row = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    if (row >= env.n_rows) return;
    const int j0 = B::first(sub);
    float hb[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
        hb[c] = j0 + c < HO::NOUT ? env.head_scratch[row * HO::NH + j0 + c] : 0.0f;
    const float hv = env.head_scratch[row * HO::NH + HO::NOUT];
    const RngKey key = rng_key(env);
    const uint32_t t = step_base(env) + (uint32_t)step;
    const float log_std = (E::NACT == 0 && pol.log_std) ? pol.log_std[0] : 0.0f;
    float logp;
    const Act<E> a = choose<E, G, C>(hb, sub, key, t, (uint32_t)row, log_std, logp);
    if (sub == 0) {
        const size_t idx = (size_t)step * env.n_rows + row;
        tr.value[idx] = hv;
        tr.logp[idx] = logp;
        store_action<E>(tr, idx, a);
    }
}

template <class E, int G>
__device__ __forceinline__ void finish_row(const EnvArgs& env, const TrajArgs& tr, int64_t row,
                                           const float (&s)[E::SR], int step, int horizon, int sub) {
    save_state<E, G>(env, row, s, sub);
    float o[E::OD];
    E::observe(s, o);
    store_obs<E::OD, G>(env.obs_scratch + row * E::OD, o, sub);
    if (step + 1 < horizon)
        store_obs<E::OD, G>(tr.obs + ((size_t)(step + 1) * env.n_rows + row) * E::OD, o, sub);
}

// Plain step: G lanes per row, the same group code as the fused kernel.
template <class E, int G>
__global__ void __launch_bounds__(256) k_plain_step(EnvArgs env, TrajArgs tr, int step,
                                                    int horizon) {
    __shared__ float params[E::KIND == Reaction::KIND ? Reaction::PARAM_FLOATS : 1];
    EnvCtx ctx{nullptr, nullptr, 0};
    if constexpr (E::KIND == Reaction::KIND) {
        // every block stages the potential (the plain form re-reads it per launch)
        stage_params(params, env.params, threadIdx.x, blockDim.x);
        ctx.lds_params = params;
    }
    __syncthreads();
    const int sub = threadIdx.x % G;
    const int64_t row = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    if (row >= env.n_rows) return;
    if constexpr (E::KIND == Reaction::KIND) {
        // the row's cache in place in the state block (each lane its own entries)
        ctx.cache = env.cache + row;
        ctx.cache_stride = (int)env.n_rows;
    }
    const RngKey key = rng_key(env);
    const uint32_t t = step_base(env) + (uint32_t)step;
    float s[E::SR];
    load_state<E>(env, row, s);
    const size_t idx = (size_t)step * env.n_rows + row;
    const Act<E> a = load_action<E>(tr, idx);
    float reward;
    bool done;
    E::template step<G>(s, a.index, a.value, t, (uint32_t)row, key, ctx, sub, reward, done);
    if (done) E::reset(s, key, t + 1, (uint32_t)row, ctx);
    if (sub == 0) {
        tr.reward[idx] = reward;
        tr.done[idx] = done ? 1 : 0;
    }
    finish_row<E, G>(env, tr, row, s, step, horizon, sub);
}

// Market step: one workgroup per tile of whole envs, exact integer sums.
__global__ void __launch_bounds__(256) k_plain_step_market(EnvArgs env, TrajArgs tr, int step,
                                                           int horizon) {
    __shared__ int sums[256 * 2];
    const Tile tl = env.tiles[blockIdx.x];
    const int n = tl.row1 - tl.row0;
    for (int i = threadIdx.x; i < 2 * (tl.env1 - tl.env0); i += blockDim.x) sums[i] = 0;
    __syncthreads();
    int slot[2], act[2];
    for (int r = threadIdx.x, q = 0; q < 2; r += blockDim.x, ++q) {
        slot[q] = -1;
        if (r < n) {
            const int row = env.row_map[tl.row0 + r];
            slot[q] = env.slot_map[tl.row0 + r];
            act[q] = static_cast<const uint8_t*>(tr.action)[(size_t)step * env.n_rows + row];
            int dh, s18;
            Market::decide(act[q], dh, s18);
            atomicAdd(&sums[slot[q] * 2], dh);
            atomicAdd(&sums[slot[q] * 2 + 1], s18);
        }
    }
    __syncthreads();
    for (int r = threadIdx.x, q = 0; q < 2; r += blockDim.x, ++q) {
        if (slot[q] < 0) continue;
        const int64_t row = env.row_map[tl.row0 + r];
        float s[Market::SD];
        load_state<Market>(env, row, s);
        float reward;
        Market::settle(s, act[q], sums[slot[q] * 2], sums[slot[q] * 2 + 1], reward);
        const size_t idx = (size_t)step * env.n_rows + row;
        tr.reward[idx] = reward;
        tr.done[idx] = 0;
        finish_row<Market, 1>(env, tr, row, s, step, horizon, 0);
    }
}

template <class E>
__global__ void k_plain_last(EnvArgs env, TrajArgs tr) {
    using HO = HeadOf<E>;
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= env.n_rows) return;
    tr.last_value[row] = env.head_scratch[row * HO::NH + HO::NOUT];
}

// The device copy of the step counter and the reset epoch that graph-captured
// launches read.
__global__ void k_set_step(uint32_t* p, uint32_t step, uint32_t epoch) {
    p[0] = step;
    p[1] = epoch;
}

// -------------------------------------------------------- small kernels --
__global__ void k_quantize(int dtype, float scale, const float* x, float* y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = x[i];
    if (dtype == DT_BF16) {
        y[i] = bf16_bits_to_f32(pack_bf16x2(v, 0.0f) & 0xFFFFu);
    } else if (dtype == DT_FP8) {
        y[i] = fp8_code_to_f32(pack_fp8x4(v / scale, 0.f, 0.f, 0.f) & 0xFFu) * scale;
    } else {
        y[i] = v;
    }
}

// ---------------------------------------------------------- dispatching --
// (env, dtype, hidden, waves, row tiles of 16, head split-M, min waves per SIMD)
#define WSX_VARIANTS(X)                      \
    X(CartPole, DT_F32, 64, 4, 1, 0, 1)      \
    X(CartPole, DT_F32, 64, 4, 2, 0, 1)      \
    X(CartPole, DT_F32, 64, 4, 4, 0, 1)      \
    X(CartPole, DT_F32, 64, 4, 1, 0, 2)      \
    X(Pendulum, DT_BF16, 256, 4, 2, 0, 1)    \
    X(Pendulum, DT_BF16, 256, 4, 4, 0, 1)    \
    X(Pendulum, DT_BF16, 256, 4, 5, 0, 1)    \
    X(Pendulum, DT_BF16, 256, 4, 2, 0, 2)    \
    X(Pendulum, DT_BF16, 256, 4, 3, 0, 2)    \
    X(Pendulum, DT_BF16, 256, 8, 2, 0, 2)    \
    X(Pendulum, DT_BF16, 256, 8, 3, 0, 2)    \
    X(Pendulum, DT_BF16, 256, 8, 4, 0, 2)    \
    X(Pendulum, DT_BF16, 256, 8, 5, 0, 2)    \
    X(Acrobot, DT_BF16, 256, 4, 2, 0, 1)     \
    X(Acrobot, DT_BF16, 256, 4, 4, 0, 1)     \
    X(Acrobot, DT_BF16, 256, 4, 5, 0, 1)     \
    X(Acrobot, DT_BF16, 256, 4, 2, 0, 2)     \
    X(Acrobot, DT_BF16, 256, 4, 3, 0, 2)     \
    X(Acrobot, DT_BF16, 256, 8, 2, 0, 2)     \
    X(Acrobot, DT_BF16, 256, 8, 3, 0, 2)     \
    X(Acrobot, DT_BF16, 256, 8, 4, 0, 2)     \
    X(Acrobot, DT_BF16, 256, 8, 5, 0, 2)     \
    X(Market, DT_BF16, 256, 4, 8, 1, 1)      \
    X(Market, DT_BF16, 256, 8, 8, 1, 2)      \
    X(Reaction, DT_FP8, 512, 4, 1, 0, 1)     \
    X(Reaction, DT_FP8, 512, 8, 1, 0, 2)     \
    X(Reaction, DT_FP8, 512, 8, 2, 0, 2)     \
    X(Reaction, DT_FP8, 512, 8, 4, 1, 2)

struct VariantEntry {
    Variant v;
    const void* fused;
    const void* policy;
    const void* trace;    // the policy kernel that also writes its hidden-layer codes
    const void* sample;   // plain-form sampling and step kernels with the same
    const void* step;     // lanes per row as the fused kernel
    int lanes;
};

template <class E, int G>
const void* step_entry() {
    if constexpr (E::KIND == Market::KIND)
        return reinterpret_cast<const void*>(&k_plain_step_market);
    else
        return reinterpret_cast<const void*>(&k_plain_step<E, G>);
}

#define WSX_G(E, NW, NT) lanes_per_row(16 * (NT), 64 * (NW), E::LANES)
#define WSX_ENTRY(E, DT, H, NW, NT, HS, OCC)                                          \
    {{E::KIND, DT, H, NW, 16 * NT, OCC, 0},                                           \
     reinterpret_cast<const void*>(&k_fused<E, E, DT, H, NW, NT, HS, OCC>),           \
     reinterpret_cast<const void*>(&k_plain_policy<E, DT, H, NW, NT, HS, OCC>),       \
     reinterpret_cast<const void*>(&k_policy_trace<E, DT, H, NW, NT, HS, OCC>),       \
     reinterpret_cast<const void*>(&k_plain_sample<E, WSX_G(E, NW, NT)>),             \
     step_entry<E, WSX_G(E, NW, NT)>(), WSX_G(E, NW, NT)},

// Fused kernels over tiles of two kinds with the same policy shape (one
// launch for a Pendulum set and an Acrobot set).
#define WSX_PAIR_VARIANTS(X)                                 \
    X(Pendulum, Acrobot, DT_BF16, 256, 4, 2, 0, 2)          \
    X(Pendulum, Acrobot, DT_BF16, 256, 4, 3, 0, 2)          \
    X(Pendulum, Acrobot, DT_BF16, 256, 4, 5, 0, 1)          \
    X(Pendulum, Acrobot, DT_BF16, 256, 8, 3, 0, 2)          \
    X(Pendulum, Acrobot, DT_BF16, 256, 8, 4, 0, 2)          \
    X(Pendulum, Acrobot, DT_BF16, 256, 8, 5, 0, 2)

#define WSX_PAIR_ENTRY(E, E2, DT, H, NW, NT, HS, OCC)                                 \
    {{E::KIND, DT, H, NW, 16 * NT, OCC, E2::KIND},                                    \
     reinterpret_cast<const void*>(&k_fused<E, E2, DT, H, NW, NT, HS, OCC>), nullptr,  \
     nullptr, nullptr, nullptr, 0},

// The row-per-wave form of the FP32 64-wide policy (one wave, one row per
// tile).
#define WSX_RW_ENTRY(E, H)                                                             \
    {{E::KIND, DT_F32, H, 1, 1, 1, 0},                                                \
     reinterpret_cast<const void*>(&k_fused_rw<E, H>),                                \
     reinterpret_cast<const void*>(&k_plain_policy_rw<E, H>),                         \
     reinterpret_cast<const void*>(&k_policy_trace_rw<E, H>),                         \
     reinterpret_cast<const void*>(&k_plain_sample<E, 1>), step_entry<E, 1>(), 1},

static const VariantEntry kVariants[] = {WSX_VARIANTS(WSX_ENTRY)
                                             WSX_PAIR_VARIANTS(WSX_PAIR_ENTRY)
                                                 WSX_RW_ENTRY(CartPole, 64)};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int n_variants() { return kNumVariants; }
const Variant& variant(int i) { return kVariants[i].v; }

static const VariantEntry* find_entry(const Variant& v) {
    for (int i = 0; i < kNumVariants; ++i) {
        const Variant& w = kVariants[i].v;
        if (w.kind == v.kind && w.dtype == v.dtype && w.hidden == v.hidden && w.waves == v.waves &&
            w.tile_rows == v.tile_rows && w.occupancy == v.occupancy && w.kind2 == v.kind2)
            return &kVariants[i];
    }
    return nullptr;
}

int fused_blocks_per_cu(const Variant& v) {
    if (v.kind >= kUserKindBase) return user_blocks_per_cu(v);
    const VariantEntry* e = find_entry(v);
    if (!e) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, e->fused, v.waves * 64, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

hipError_t launch_fused(const Variant& v, const Batch& batch, int grid, hipStream_t s) {
    if (v.kind >= kUserKindBase) return launch_user_fused(v, batch, grid, s);
    const VariantEntry* e = find_entry(v);
    if (!e) return hipErrorInvalidValue;
    void* args[] = {(void*)&batch};
    return hipLaunchKernel(e->fused, dim3(grid), dim3(v.waves * 64), args, 0, s);
}

template <class E>
static hipError_t plain_sequence(const VariantEntry* e, const EnvArgs& env, const PolicyArgs& pol,
                                 const TrajArgs& tr, int horizon, hipStream_t s) {
    const int threads = 256;
    const int blocks = (int)((env.n_rows + threads - 1) / threads);
    const int rows_per_block = threads / e->lanes;
    const int gblocks = (int)((env.n_rows + rows_per_block - 1) / rows_per_block);
    hipLaunchKernelGGL(k_plain_observe<E>, dim3(blocks), dim3(threads), 0, s, env, tr, horizon);
    void* pargs[] = {(void*)&env, (void*)&pol};
    for (int step = 0; step <= horizon; ++step) {
        hipError_t err = hipLaunchKernel(e->policy, dim3(env.n_tiles), dim3(e->v.waves * 64),
                                         pargs, 0, s);
        if (err != hipSuccess) return err;
        if (step == horizon) break;
        void* sargs[] = {(void*)&env, (void*)&pol, (void*)&tr, (void*)&step};
        err = hipLaunchKernel(e->sample, dim3(gblocks), dim3(threads), sargs, 0, s);
        if (err != hipSuccess) return err;
        void* targs[] = {(void*)&env, (void*)&tr, (void*)&step, (void*)&horizon};
        if constexpr (E::KIND == Market::KIND)
            err = hipLaunchKernel(e->step, dim3(env.n_tiles), dim3(256), targs, 0, s);
        else
            err = hipLaunchKernel(e->step, dim3(gblocks), dim3(threads), targs, 0, s);
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_plain_last<E>, dim3(blocks), dim3(threads), 0, s, env, tr);
    return hipGetLastError();
}

hipError_t launch_plain(const Variant& v, const EnvArgs& env, const PolicyArgs& pol,
                        const TrajArgs& tr, int horizon, bool, hipStream_t s) {
    const VariantEntry* e = find_entry(v);
    if (!e) return hipErrorInvalidValue;
    switch (v.kind) {
    case CartPole::KIND: return plain_sequence<CartPole>(e, env, pol, tr, horizon, s);
    case Pendulum::KIND: return plain_sequence<Pendulum>(e, env, pol, tr, horizon, s);
    case Acrobot::KIND: return plain_sequence<Acrobot>(e, env, pol, tr, horizon, s);
    case Market::KIND: return plain_sequence<Market>(e, env, pol, tr, horizon, s);
    case Reaction::KIND: return plain_sequence<Reaction>(e, env, pol, tr, horizon, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_set_step(uint32_t* step_ptr, uint32_t step, uint32_t epoch, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, step_ptr, step, epoch);
    return hipGetLastError();
}

hipError_t launch_reset(int kind, const EnvArgs& env, hipStream_t s) {
    const int threads = 256;
    const int blocks = (int)((env.n_rows + threads - 1) / threads);
    switch (kind) {
    case CartPole::KIND: hipLaunchKernelGGL(k_reset<CartPole>, dim3(blocks), dim3(threads), 0, s, env); break;
    case Pendulum::KIND: hipLaunchKernelGGL(k_reset<Pendulum>, dim3(blocks), dim3(threads), 0, s, env); break;
    case Acrobot::KIND: hipLaunchKernelGGL(k_reset<Acrobot>, dim3(blocks), dim3(threads), 0, s, env); break;
    case Market::KIND: hipLaunchKernelGGL(k_reset<Market>, dim3(blocks), dim3(threads), 0, s, env); break;
    case Reaction::KIND: hipLaunchKernelGGL(k_reset<Reaction>, dim3(blocks), dim3(threads), 0, s, env); break;
    default: return launch_user_reset(kind, env, s);
    }
    return hipGetLastError();
}

hipError_t launch_policy_forward(const Variant& v, const PolicyArgs& pol, const float* obs,
                                 int64_t rows, float* head, hipStream_t s) {
    const VariantEntry* e = find_entry(v);
    if (!e) return hipErrorInvalidValue;
    EnvArgs env{};
    env.obs_scratch = const_cast<float*>(obs);
    env.head_scratch = head;
    env.n_rows = rows;
    env.tile_rows = v.tile_rows;
    env.n_tiles = (int)((rows + v.tile_rows - 1) / v.tile_rows);
    void* args[] = {(void*)&env, (void*)&pol};
    return hipLaunchKernel(e->policy, dim3(env.n_tiles), dim3(v.waves * 64), args, 0, s);
}

hipError_t launch_policy_trace(const Variant& v, const PolicyArgs& pol, const float* obs,
                               int64_t rows, float* head, void* act1, void* act2, hipStream_t s) {
    const VariantEntry* e = find_entry(v);
    if (!e || !e->trace) return hipErrorInvalidValue;
    EnvArgs env{};
    env.obs_scratch = const_cast<float*>(obs);
    env.head_scratch = head;
    env.n_rows = rows;
    env.tile_rows = v.tile_rows;
    env.n_tiles = (int)((rows + v.tile_rows - 1) / v.tile_rows);
    char* a1 = static_cast<char*>(act1);
    char* a2 = static_cast<char*>(act2);
    void* args[] = {(void*)&env, (void*)&pol, (void*)&a1, (void*)&a2};
    return hipLaunchKernel(e->trace, dim3(env.n_tiles), dim3(v.waves * 64), args, 0, s);
}

hipError_t launch_quantize(int dtype, float scale, const float* x, float* y, int64_t n,
                           hipStream_t s) {
    const int threads = 256;
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                       s, dtype, scale, x, y, n);
    return hipGetLastError();
}

}  // namespace wsx
