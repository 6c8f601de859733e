// returns.hip -- discounted returns and GAE advantages on the device, FP64
// (arXiv 2408.00930, Sec. 3: actor-critic training consumes them; GAE of
// Schulman et al. 2016).
//
// Four kernels, chosen by the set's shape in launch_returns. For sets with
// few rows and horizons of at most 32 steps, a time-parallel scan: both
// recursions are affine maps run backwards in time,
//   A_t = delta_t + gamma lambda (1 - d_t) A_{t+1},  G_t = r_t + gamma (1 - d_t) G_{t+1},
// so a block of consecutive steps composes into one map x -> b + c x with
// (c1, b1) o (c2, b2) = (c1 c2, b1 + c1 b2). A workgroup owns 32 rows and
// walks the horizon backwards in tiles of 64 steps: the tile is loaded
// coalesced (consecutive rows adjacent) into LDS; each wave then takes a row
// with one step per lane and forms the suffix compositions of the tile with a
// Hillis-Steele scan over wavefront shuffles (6 rounds of 64-bit shuffles),
// applies them to the carry from the later tile, and leaves the carry of the
// tile's first step for the next (earlier) tile.
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace wsx {

constexpr int kRetRows = 32;   // rows per workgroup (128-byte rows of float)
constexpr int kRetSteps = 64;  // steps per tile = lanes of a wave
// sets with at least this many rows per CU take the row-parallel kernel
// unless their horizon fits eight one-block segments
constexpr int kRowsPerLaneMin = 24;

__global__ void __launch_bounds__(256)
k_returns(const float* __restrict__ reward, const float* __restrict__ value,
          const uint8_t* __restrict__ done, const float* __restrict__ last_value, int T,
          int64_t rows, double gamma, double lambda, int bootstrap, void* ret, void* adv,
          int out_f64) {
    __shared__ float s_r[kRetSteps][kRetRows + 1];
    __shared__ float s_v[kRetSteps][kRetRows + 1];
    __shared__ uint8_t s_d[kRetSteps][kRetRows + 4];
    __shared__ double s_g[kRetSteps][kRetRows + 1];
    __shared__ double s_a[kRetSteps][kRetRows + 1];
    __shared__ double carry_g[kRetRows], carry_a[kRetRows], carry_v[kRetRows];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * kRetRows;
    if (tid < kRetRows) {
        const int64_t r = row0 + tid;
        const double vT = (bootstrap && r < rows) ? (double)last_value[r] : 0.0;
        carry_g[tid] = vT;   // G_T
        carry_a[tid] = 0.0;  // A_T
        carry_v[tid] = vT;   // V_T
    }
    const double gl = gamma * lambda;
    const int n_tiles = (T + kRetSteps - 1) / kRetSteps;
    for (int tt = n_tiles - 1; tt >= 0; --tt) {
        const int tbase = tt * kRetSteps;
        const int tlen = min(kRetSteps, T - tbase);
        __syncthreads();   // previous tile's outputs have been stored
        for (int i = tid; i < kRetSteps * kRetRows; i += 256) {
            const int t = i / kRetRows, j = i % kRetRows;
            const int64_t r = row0 + j;
            if (t < tlen && r < rows) {
                const size_t g = (size_t)(tbase + t) * rows + r;
                s_r[t][j] = reward[g];
                s_v[t][j] = value[g];
                s_d[t][j] = done[g];
            } else {
                s_r[t][j] = 0.0f;
                s_v[t][j] = 0.0f;
                s_d[t][j] = 0;
            }
        }
        __syncthreads();
        for (int j = wave; j < kRetRows; j += 4) {
            const int t = lane;
            const bool live = t < tlen;
            const double r = s_r[t][j];
            const double v = s_v[t][j];
            const double keep = s_d[t][j] ? 0.0 : 1.0;
            double v_next = __shfl_down(v, 1);
            const double ca_in = carry_a[j], cg_in = carry_g[j], cv_in = carry_v[j];
            if (t == tlen - 1) v_next = cv_in;
            // this step's maps; steps past the horizon are the identity
            double ca = live ? gl * keep : 1.0;
            double ba = live ? r + gamma * keep * v_next - v : 0.0;
            double cg = live ? gamma * keep : 1.0;
            double bg = live ? r : 0.0;
#pragma unroll
            for (int off = 1; off < kRetSteps; off <<= 1) {
                const double ca2 = __shfl_down(ca, off), ba2 = __shfl_down(ba, off);
                const double cg2 = __shfl_down(cg, off), bg2 = __shfl_down(bg, off);
                if (lane + off < kRetSteps) {
                    ba = ba + ca * ba2;
                    ca = ca * ca2;
                    bg = bg + cg * bg2;
                    cg = cg * cg2;
                }
            }
            const double a = ba + ca * ca_in;
            const double g = bg + cg * cg_in;
            s_a[t][j] = a;
            s_g[t][j] = g;
            if (lane == 0) {
                carry_a[j] = a;
                carry_g[j] = g;
                carry_v[j] = v;
            }
        }
        __syncthreads();
        for (int i = tid; i < kRetSteps * kRetRows; i += 256) {
            const int t = i / kRetRows, j = i % kRetRows;
            const int64_t r = row0 + j;
            if (t < tlen && r < rows) {
                const size_t g = (size_t)(tbase + t) * rows + r;
                if (out_f64) {
                    static_cast<double*>(ret)[g] = s_g[t][j];
                    static_cast<double*>(adv)[g] = s_a[t][j];
                } else {
                    static_cast<float*>(ret)[g] = (float)s_g[t][j];
                    static_cast<float*>(adv)[g] = (float)s_a[t][j];
                }
            }
        }
    }
}

// Row-parallel form for sets with many rows: lane = row, the recursion run
// backwards over the horizon in registers (the same FP64 operations as one
// step of the scan), loads and stores coalesced over consecutive rows. A set
// of 10,000 rows is only ~160 waves, too few to hide HBM latency by
// occupancy, so each lane keeps the next block of kRowBlock steps' loads in
// flight while it runs the current block. With rows >= 64 waves' worth this
// keeps every CU streaming, where the time-parallel scan above would stage
// each 64-step tile through LDS.
constexpr int kRowBlock = 16;

template <int OUT_F64>
__global__ void __launch_bounds__(64)
k_returns_rows(const float* __restrict__ reward, const float* __restrict__ value,
               const uint8_t* __restrict__ done, const float* __restrict__ last_value, int T,
               int64_t rows, double gamma, double lambda, int bootstrap, void* __restrict__ ret,
               void* __restrict__ adv) {
    const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (r >= rows) return;
    const double gl = gamma * lambda;
    const double vT = bootstrap ? (double)last_value[r] : 0.0;
    double g = vT, a = 0.0, v_next = vT;
    // a block holds steps t_hi, t_hi - 1, ..., t_hi - kRowBlock + 1; only the
    // last (lowest) block of the horizon may be partial (FULL false: steps
    // below 0 are skipped)
    float rw[2][kRowBlock], vv[2][kRowBlock];
    uint8_t dd[2][kRowBlock];
    auto load = [&](auto full, int t_hi, int buf) {
#pragma unroll
        for (int j = 0; j < kRowBlock; ++j) {
            const int t = t_hi - j;
            if (decltype(full)::value || t >= 0) {
                const size_t i = (size_t)t * rows + r;
                rw[buf][j] = reward[i];
                vv[buf][j] = value[i];
                dd[buf][j] = done[i];
            }
        }
    };
    auto run = [&](auto full, int t_hi, int buf) {
#pragma unroll
        for (int j = 0; j < kRowBlock; ++j) {
            const int t = t_hi - j;
            if (decltype(full)::value || t >= 0) {
                const size_t i = (size_t)t * rows + r;
                const double rt = rw[buf][j], v = vv[buf][j];
                const double keep = dd[buf][j] ? 0.0 : 1.0;
                a = (rt + gamma * keep * v_next - v) + gl * keep * a;
                g = rt + gamma * keep * g;
                v_next = v;
                if (OUT_F64) {
                    static_cast<double*>(ret)[i] = g;
                    static_cast<double*>(adv)[i] = a;
                } else {
                    static_cast<float*>(ret)[i] = (float)g;
                    static_cast<float*>(adv)[i] = (float)a;
                }
            }
        }
    };
    const std::true_type full{};
    const std::false_type part{};
    const int nb = T / kRowBlock;   // full blocks, from the end of the horizon
    const int rem = T - nb * kRowBlock;
    if (nb > 0) load(full, T - 1, 0);
    // two blocks per iteration so the buffers keep fixed registers; the next
    // block's loads are issued before the current block's recursion
    for (int k = 0; k < nb; k += 2) {
        if (k + 1 < nb) load(full, T - 1 - (k + 1) * kRowBlock, 1);
        run(full, T - 1 - k * kRowBlock, 0);
        if (k + 1 >= nb) break;
        if (k + 2 < nb) load(full, T - 1 - (k + 2) * kRowBlock, 0);
        run(full, T - 1 - (k + 1) * kRowBlock, 1);
    }
    if (rem > 0) {   // steps rem - 1 .. 0
        load(part, rem - 1, 0);
        run(part, rem - 1, 0);
    }
}

// Segmented row-parallel form for horizons of 33 to 16 x 32 steps: a
// workgroup owns 64 rows (lane = row) and one wave per 32-step segment of
// the horizon. Each wave loads its segment into registers once
// (branch-free: indices past the set are clamped and their values unused),
// composes its steps' affine maps backwards (G_start = bg + cg G_end,
// A_start = ba + ca A_end; the A map's last step takes V at the next
// segment's first step), publishes (cg, bg, ca, ba) in LDS, forms its carry
// from the later segments' maps, and runs the same recursion as
// k_returns_rows from its registers to write the outputs. A row's chain of
// dependent loads is one segment long instead of the whole horizon.
// Up to 16 segments (1024 threads, four waves per SIMD within 128 VGPRs).
constexpr int kSeg = 32;
constexpr int kSegMax = 16;

template <int OUT_F64>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64 * kSegMax)))
k_returns_seg(const float* __restrict__ reward, const float* __restrict__ value,
              const uint8_t* __restrict__ done, const float* __restrict__ last_value, int T,
              int64_t rows, double gamma, double lambda, int bootstrap, void* __restrict__ ret,
              void* __restrict__ adv) {
    __shared__ double maps[4][kSegMax][64];   // cg, bg, ca, ba per segment and row
    // Element offsets fit 32 bits (the launcher takes this form only while
    // rows x T < 2^31). The segment index is wave-uniform: held in a scalar
    // register it keeps each step's offset scalar, so a lane holds one vector
    // offset (its row) instead of one per step.
    const int lane = threadIdx.x & 63, nseg = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nrows = (uint32_t)rows;
    const uint32_t r = blockIdx.x * 64u + (uint32_t)lane;
    const bool ok = r < nrows;
    const uint32_t rl = ok ? r : nrows - 1;   // a row inside the set, for the loads
    const double gl = gamma * lambda;
    const int t0 = w * kSeg;   // this wave's steps t0 .. t0 + kSeg - 1 (below T)
    float rw[kSeg], vv[kSeg];
    uint32_t dmask = 0;   // bit j: step t0 + j terminated
#pragma unroll
    for (int j = 0; j < kSeg; ++j)
        dmask |= (uint32_t)(done[(uint32_t)min(t0 + j, T - 1) * nrows + rl] != 0) << j;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const uint32_t i = (uint32_t)min(t0 + j, T - 1) * nrows + rl;
        rw[j] = reward[i];
        vv[j] = value[i];
    }
    const int t_end = min(t0 + kSeg, T);   // first step after the segment
    const double v_T = bootstrap ? (double)last_value[rl] : 0.0;
    // V at the segment's end: the next segment's first value, or V(s_T)
    const double v_end = t_end < T ? (double)value[(uint32_t)t_end * nrows + rl] : v_T;
    double cg = 1.0, bg = 0.0, ca = 1.0, ba = 0.0, v_next = v_end;
#pragma unroll
    for (int j = kSeg - 1; j >= 0; --j) {
        if (t0 + j < T) {
            const double rt = rw[j], v = vv[j];
            const double keep = (dmask >> j) & 1u ? 0.0 : 1.0;
            ba = (rt + gamma * keep * v_next - v) + gl * keep * ba;
            ca = gl * keep * ca;
            bg = rt + gamma * keep * bg;
            cg = gamma * keep * cg;
            v_next = v;
        }
    }
    maps[0][w][lane] = cg;
    maps[1][w][lane] = bg;
    maps[2][w][lane] = ca;
    maps[3][w][lane] = ba;
    __syncthreads();
    // carry into this segment: the later segments' maps applied to (G_T, A_T)
    double g = v_T, a = 0.0;
    for (int k = nseg - 1; k > w; --k) {
        g = maps[1][k][lane] + maps[0][k][lane] * g;
        a = maps[3][k][lane] + maps[2][k][lane] * a;
    }
    if (!ok) return;
    v_next = v_end;
#pragma unroll
    for (int j = kSeg - 1; j >= 0; --j) {
        const int t = t0 + j;
        if (t < T) {
            const uint32_t i = (uint32_t)t * nrows + r;
            const double rt = rw[j], v = vv[j];
            const double keep = (dmask >> j) & 1u ? 0.0 : 1.0;
            a = (rt + gamma * keep * v_next - v) + gl * keep * a;
            g = rt + gamma * keep * g;
            v_next = v;
            if (OUT_F64) {
                static_cast<double*>(ret)[i] = g;
                static_cast<double*>(adv)[i] = a;
            } else {
                static_cast<float*>(ret)[i] = (float)g;
                static_cast<float*>(adv)[i] = (float)a;
            }
        }
    }
}

// Long horizons (past 512 steps): the same with segments of nsub blocks of
// kSegL steps. Each block is loaded into registers in the first pass and
// again (from L2) in the second, so a lane's registers hold one block
// whatever the segment's length (half the short form's block, as the running
// maps stay live across the loads).
constexpr int kSegL = 16;   // steps per block of the long form

template <int OUT_F64>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64 * kSegMax)))
k_returns_seg_long(const float* __restrict__ reward, const float* __restrict__ value,
                   const uint8_t* __restrict__ done, const float* __restrict__ last_value, int T,
                   int nsub, int64_t rows, double gamma, double lambda, int bootstrap,
                   void* __restrict__ ret, void* __restrict__ adv) {
    __shared__ double maps[4][kSegMax][64];   // cg, bg, ca, ba per segment and row
    // Element offsets fit 32 bits (the launcher takes this form only while
    // rows x T < 2^31). The segment index is wave-uniform: held in a scalar
    // register it keeps each step's offset scalar, so a lane holds one vector
    // offset (its row) instead of one per step.
    const int lane = threadIdx.x & 63, nseg = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nrows = (uint32_t)rows;
    const uint32_t r = blockIdx.x * 64u + (uint32_t)lane;
    const bool ok = r < nrows;
    const uint32_t rl = ok ? r : nrows - 1;   // a row inside the set, for the loads
    const double gl = gamma * lambda;
    // this wave's steps ts .. te - 1: nsub blocks of kSegL steps (ts below T)
    const int ts = w * kSegL * nsub, te = min(ts + kSegL * nsub, T);
    float rw[kSegL], vv[kSegL];
    uint32_t dmask = 0;   // bit j: step t0 + j terminated (j < 16)
    auto load = [&](int t0) {
        dmask = 0;
#pragma unroll
        for (int j = 0; j < kSegL; ++j)
            dmask |= (uint32_t)(done[(uint32_t)min(t0 + j, T - 1) * nrows + rl] != 0) << j;
#pragma unroll
        for (int j = 0; j < kSegL; ++j) {
            const uint32_t i = (uint32_t)min(t0 + j, T - 1) * nrows + rl;
            rw[j] = reward[i];
            vv[j] = value[i];
        }
    };
    const double v_T = bootstrap ? (double)last_value[rl] : 0.0;
    // V at the segment's end: the next segment's first value, or V(s_T)
    const double v_end = te < T ? (double)value[(uint32_t)te * nrows + rl] : v_T;
    double cg = 1.0, bg = 0.0, ca = 1.0, ba = 0.0, v_next = v_end;
    // the segment's map, composed backwards block by block
#pragma nounroll
    for (int b = nsub - 1; b >= 0; --b) {
        const int t0 = ts + b * kSegL;
        if (t0 >= te) continue;
        load(t0);
#pragma unroll
        for (int j = kSegL - 1; j >= 0; --j) {
            if (t0 + j < te) {
                const double rt = rw[j], v = vv[j];
                const double keep = (dmask >> j) & 1u ? 0.0 : 1.0;
                ba = (rt + gamma * keep * v_next - v) + gl * keep * ba;
                ca = gl * keep * ca;
                bg = rt + gamma * keep * bg;
                cg = gamma * keep * cg;
                v_next = v;
            }
        }
    }
    maps[0][w][lane] = cg;
    maps[1][w][lane] = bg;
    maps[2][w][lane] = ca;
    maps[3][w][lane] = ba;
    __syncthreads();
    // carry into this segment: the later segments' maps applied to (G_T, A_T)
    double g = v_T, a = 0.0;
    for (int k = nseg - 1; k > w; --k) {
        g = maps[1][k][lane] + maps[0][k][lane] * g;
        a = maps[3][k][lane] + maps[2][k][lane] * a;
    }
    if (!ok) return;
    v_next = v_end;
#pragma nounroll
    for (int b = nsub - 1; b >= 0; --b) {
        const int t0 = ts + b * kSegL;
        if (t0 >= te) continue;
        load(t0);   // again: an L2 hit
#pragma unroll
        for (int j = kSegL - 1; j >= 0; --j) {
            const int t = t0 + j;
            if (t < te) {
                const uint32_t i = (uint32_t)t * nrows + r;
                const double rt = rw[j], v = vv[j];
                const double keep = (dmask >> j) & 1u ? 0.0 : 1.0;
                a = (rt + gamma * keep * v_next - v) + gl * keep * a;
                g = rt + gamma * keep * g;
                v_next = v;
                if (OUT_F64) {
                    static_cast<double*>(ret)[i] = g;
                    static_cast<double*>(adv)[i] = a;
                } else {
                    static_cast<float*>(ret)[i] = (float)g;
                    static_cast<float*>(adv)[i] = (float)a;
                }
            }
        }
    }
}

hipError_t launch_returns(const float* reward, const float* value, const uint8_t* done,
                          const float* last_value, int horizon, int64_t rows, double gamma,
                          double lambda, int bootstrap, void* ret, void* adv, int out_f64,
                          hipStream_t s) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the segmented forms while one chain per row leaves the set latency-bound
    // (below one 64-row wave per CU): up to 16 segments of one 32-step block,
    // past 512 steps up to 16 segments of nsub 16-step blocks. From 24 rows
    // per CU up they are kept to horizons of 8 segments, past which the row
    // form is as fast; with more rows the row form streams faster, and the
    // time-parallel scan takes the rest (horizons within one block, or
    // offsets past 32 bits)
    const int64_t nblk = ((int64_t)horizon + kSeg - 1) / kSeg;
    const bool many = rows >= (int64_t)kRowsPerLaneMin * cus;
    if (rows < (int64_t)64 * cus && horizon > kSeg && rows * horizon < ((int64_t)1 << 31) &&
        (!many || nblk <= 8)) {
        const dim3 grid((unsigned)((rows + 63) / 64));
        if (nblk > kSegMax) {
            const int64_t nb16 = ((int64_t)horizon + kSegL - 1) / kSegL;
            const int nsub = (int)((nb16 + kSegMax - 1) / kSegMax);
            const dim3 block(64 * (int)((nb16 + nsub - 1) / nsub));
            auto* k = out_f64 ? k_returns_seg_long<1> : k_returns_seg_long<0>;
            hipLaunchKernelGGL(k, grid, block, 0, s, reward, value, done, last_value, horizon,
                               nsub, rows, gamma, lambda, bootstrap, ret, adv);
        } else {
            const dim3 block(64 * (int)nblk);
            auto* k = out_f64 ? k_returns_seg<1> : k_returns_seg<0>;
            hipLaunchKernelGGL(k, grid, block, 0, s, reward, value, done, last_value, horizon,
                               rows, gamma, lambda, bootstrap, ret, adv);
        }
        return hipGetLastError();
    }
    if (rows >= (int64_t)kRowsPerLaneMin * cus) {
        const unsigned blocks = (unsigned)((rows + 63) / 64);
        if (out_f64)
            hipLaunchKernelGGL(k_returns_rows<1>, dim3(blocks), dim3(64), 0, s, reward, value, done,
                               last_value, horizon, rows, gamma, lambda, bootstrap, ret, adv);
        else
            hipLaunchKernelGGL(k_returns_rows<0>, dim3(blocks), dim3(64), 0, s, reward, value, done,
                               last_value, horizon, rows, gamma, lambda, bootstrap, ret, adv);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)((rows + kRetRows - 1) / kRetRows);
    hipLaunchKernelGGL(k_returns, dim3(blocks), dim3(256), 0, s, reward, value, done, last_value,
                       horizon, rows, gamma, lambda, bootstrap, ret, adv, out_f64);
    return hipGetLastError();
}

}  // namespace wsx
