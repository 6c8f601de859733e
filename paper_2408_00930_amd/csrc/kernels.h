// kernels.h -- kernel argument blocks and host-side launcher declarations
// shared by the roll-out kernels (rollout.hip, returns.hip) and the C-ABI
// layer (abi.cpp). Internal to the library.
#pragma once

#ifndef __HIPCC_RTC__   // the run-time compiler provides the runtime itself
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace wsx {

struct PolicyArgs {
    const void* w1;
    const void* w2;
    const void* w3;
    const float* b1;
    const float* b2;
    const float* b3;
    const float* s1;  // FP8 row scales (NULL otherwise)
    const float* s2;
    const float* s3;
    const float* log_std;
    float act_scale[3];
    int32_t d_in, hidden, n_head;
};

struct TrajArgs {
    float* obs;
    void* action;
    float* reward;
    uint8_t* done;
    float* value;
    float* logp;
    float* last_value;
};

// Tile of a workgroup: rows [row0, row1) of envs [env0, env1). For the market
// (tiles packed from whole envs in any order) [row0, row1) is a range of the
// row map: entry i holds the global row of tile slot i - row0, and the slot
// map the index of that row's env among the tile's env1 - env0 envs.
struct Tile {
    int32_t row0, row1, env0, env1;
};

struct EnvArgs {
    int32_t kind;             // environment kind (WSX_CARTPOLE ...)
    float* state;             // SoA [state_dim][n_rows]
    float* obs_scratch;       // [n_rows][obs_dim]    (plain mode)
    float* head_scratch;      // [n_rows][n_head]     (plain mode)
    const float* params;      // reaction potential block (global)
    const int32_t* offsets;   // market CSR offsets [n_envs + 1]
    const Tile* tiles;        // tile table [n_tiles]
    const int32_t* row_map;   // market: global row of each tile slot [n_rows]
    const uint8_t* slot_map;  // market: the row's env among its tile's envs [n_rows]
    double* cache;            // reaction: FP64 energy terms [Reaction::NCACHE][n_rows]
    const uint32_t* step_ptr; // graph mode: device copy of [step counter, epoch]
    int64_t n_rows;
    int32_t n_envs;
    int32_t n_tiles;
    int32_t tile_rows;        // rows per tile (single-agent kinds), <= the kernel's
    uint32_t k0, k1, epoch;
    uint32_t t0;              // step counter at the start of the launch; with
                              // step_ptr, its offset from the device counter
};

// Entries of the reaction's per-row FP64 energy cache (A x, then the squared
// distances to the Gaussians' centres).
constexpr int kReactionCache = 20 + 64;

// Returns and GAE of a segment's rows, computed by the tiles of a fused
// launch after their steps ([steps][rows] outputs, offset like the
// trajectory); ret == NULL: none.
struct GaeArgs {
    void* ret;
    void* adv;
    double gamma, lambda;
    int32_t bootstrap;
    int32_t out_f64;
};

// One roll-out request inside a fused launch: its environment set, its policy,
// its trajectory pointers (offset to the launch's first slot) and its steps.
struct Segment {
    EnvArgs env;
    TrajArgs tr;
    PolicyArgs pol;
    GaeArgs gae;
    int32_t steps;
    int32_t tile_begin;   // first tile of this segment in the launch
    int32_t last;         // 1: also evaluate V(s_T) into tr.last_value after the steps
    int32_t reset;        // 1: rows start from the RESET draw of step t0 (the epoch's
                          // initial state), not from the state block
};

// The tiles of a fused launch: up to kInlineSegments segments passed with the
// launch, or a device table of them; sorted by tile_begin.
constexpr int kInlineSegments = 4;
struct Batch {
    const Segment* table;
    Segment inl[kInlineSegments];
    int32_t n_segs;
    int32_t n_tiles;
    int32_t any_reset;   // some segment has `reset` set
    int32_t any_gae;     // some segment has gae.ret set
};

// One compiled variant of the fused / plain kernels for an environment kind
// (kind2 != 0: a fused kernel that also runs tiles of a second kind with the
// same policy shape; it has no plain form).
struct Variant {
    int32_t kind, dtype, hidden, waves, tile_rows, occupancy;   // occupancy: min waves/SIMD
    int32_t kind2;
};

// Actor-critic update (update.hip). AcArgs are the kernels' arguments; the
// workspace pointers are filled in by launch_ac_grad.
struct AcArgs {
    PolicyArgs pol;
    const float* obs;        // [n][d_in]
    const void* action;      // uint8 (discrete) or float (Gaussian) [n]
    const float* ret;        // [n]
    const float* adv;        // [n]
    int64_t n;
    int32_t n_act;           // 0: Gaussian
    float value_coef, entropy_coef, inv_n;   // inv_n: 1 / all samples of the call
    bool accumulate;         // add to the workgroups' partial sums (later chunks)
    char* dz2_rows;          // workspace [n][H] in the policy format
    float* part_fwd;         // per-workgroup partial sums of the kernels
    float* part_bwd;
    float* part_w2;
};
struct AcOut {               // FP32 gradients, the policy's shapes
    float *w1, *b1, *w2, *b2, *w3, *b3, *log_std;
};
struct AcLaunch {
    AcArgs args;
    int dtype;
    void* workspace;
    int grid;                // workgroups of the two per-tile kernels
    AcOut out;
};
// Adam on several tensors in one launch (the same step and hyper-parameters).
constexpr int kAdamMaxTensors = 16;
struct AdamSeg {
    float* param;
    const float* grad;
    float *m, *v;
    int64_t n;
    void* store;   // NULL, or the parameter in store_dtype
    int store_dtype;
};
struct AdamTable {
    AdamSeg seg[kAdamMaxTensors];
};
#ifndef __HIPCC_RTC__   // host-side launchers
bool ac_supported(int dtype, int hidden, int d_in, int n_head);
// The allocation-free gradient: at most kAcStaticSamples samples, workspace in
// a file-scope device array (its per-device address, or nullptr and *err).
constexpr int64_t kAcStaticSamples = 2048;
size_t ac_static_capacity();
void* ac_static_workspace(hipError_t* err);
int64_t ac_chunk_samples(int64_t n);   // samples per chunk of a call over n
size_t ac_workspace_bytes(int dtype, int hidden, int64_t n, int grid);
hipError_t launch_ac_grad(const AcLaunch& l, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, void* store,
                       int store_dtype, hipStream_t s);
hipError_t launch_adam_many(const AdamTable& t, int n_tensors, int64_t most, float lr, float b1,
                            float b2, float eps, float c1, float c2, hipStream_t s);

// User environment kinds compiled at run time (compose.cpp): kinds
// kUserKindBase, kUserKindBase + 1, ...
constexpr int kUserKindBase = 100;
struct KindInfo;
bool user_kind_info(int kind, KindInfo& k);
bool user_variant(int kind, Variant& v);
hipError_t launch_user_fused(const Variant& v, const Batch& batch, int grid, hipStream_t s);
hipError_t launch_user_reset(int kind, const EnvArgs& env, hipStream_t s);
int user_blocks_per_cu(const Variant& v);

// Launchers (return hipError_t of the launch).
hipError_t launch_reset(int kind, const EnvArgs& env, hipStream_t s);
hipError_t launch_fused(const Variant& v, const Batch& batch, int grid, hipStream_t s);
hipError_t launch_plain(const Variant& v, const EnvArgs& env, const PolicyArgs& pol,
                        const TrajArgs& tr, int horizon, bool counter_from_device,
                        hipStream_t s);
hipError_t launch_set_step(uint32_t* step_ptr, uint32_t step, uint32_t epoch, hipStream_t s);
hipError_t launch_policy_forward(const Variant& v, const PolicyArgs& pol, const float* obs,
                                 int64_t rows, float* head, hipStream_t s);
hipError_t launch_policy_trace(const Variant& v, const PolicyArgs& pol, const float* obs,
                               int64_t rows, float* head, void* act1, void* act2, hipStream_t s);
hipError_t launch_quantize(int dtype, float scale, const float* x, float* y, int64_t n,
                           hipStream_t s);
hipError_t launch_returns(const float* reward, const float* value, const uint8_t* done,
                          const float* last_value, int horizon, int64_t rows, double gamma,
                          double lambda, int bootstrap, void* ret, void* adv, int out_f64,
                          hipStream_t s);

// The compiled variants and the workgroups of a fused launch a CU can hold.
int n_variants();
const Variant& variant(int i);
int fused_blocks_per_cu(const Variant& v);

#endif

}  // namespace wsx
