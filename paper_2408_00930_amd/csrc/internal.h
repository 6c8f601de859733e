// internal.h -- host-side pieces shared by the C-ABI layer (abi.cpp) and the
// roll-out server (serve.cpp): error reporting, per-kind shapes, the
// state-block layout and the environment handle. Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/wsx.h"
#include "kernels.h"

namespace wsx {

// Records a message for wsx_last_error() and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);

// Shapes of an environment kind and the default variant of its fused kernel.
struct KindInfo {
    int sd, od, nact, dtype, hidden, tile_rows, waves, occupancy;
};
bool kind_info(int kind, KindInfo& k);
int n_head_of(const KindInfo& k);
size_t align256(size_t x);

// Byte offsets of the parts of an environment set's device state block.
struct Layout {
    size_t state, obs, head, offsets, tiles, row_map, slot_map, cache, step, total;
};
Layout layout_of(const KindInfo& k, int64_t n_envs, int64_t n_rows, bool market,
                 bool reaction = false);

// The compiled kernel with the fewest row slots >= tile_rows; waves /
// occupancy 0 match any compiled value.
bool find_variant(int kind, int dtype, int hidden, int waves, int tile_rows, int occupancy,
                  Variant& out);

// The fused kernel over tiles of two kinds (either order), same rules.
bool find_pair_variant(int kind, int kind2, int dtype, int hidden, int waves, int tile_rows,
                       int occupancy, Variant& out);

// Packing of whole market envs into tiles (first-fit decreasing): the tile
// table, the row map and the slot map of the state block.
void pack_market_tiles(const int32_t* offsets, int64_t n_envs, int cap, std::vector<Tile>& tiles,
                       std::vector<int32_t>& row_map, std::vector<uint8_t>& slot_map);

// The autotuner's entry for an environment set, if there is one.
bool tune_lookup(int32_t kind, int64_t n_envs, int64_t n_rows, int32_t cus, wsx_tune_entry& out);

}  // namespace wsx

struct wsx_env {
    int kind;
    wsx::KindInfo info;
    int64_t n_envs, n_rows;
    uint64_t seed;
    uint32_t step, epoch;
    char* block;
    const float* params;
    wsx::Layout lay;
    int n_tiles;
    int tile_rows;
    int waves;
    int occupancy;
    int device;
    int cus;
    int chunk;   // steps per fused launch in WSX_MODE_FUSED_GRAPH (0 = horizon)
    // graph cache (the launches of one horizon, one mode)
    hipGraphExec_t graph;
    hipStream_t capture_stream;
    std::vector<char> graph_key;
};

namespace wsx {
EnvArgs env_args(const wsx_env* env);
// trajectory pointers advanced by `slots` row-steps
TrajArgs traj_at(const TrajArgs& t, const KindInfo& k, size_t slots);
PolicyArgs policy_args(const wsx_policy* p);
int check_policy(const wsx_policy* p, const KindInfo& k, int kind);
int check_traj(const wsx_env* env, const wsx_traj* traj, int32_t horizon);
TrajArgs traj_args(const wsx_traj* traj);
}  // namespace wsx
