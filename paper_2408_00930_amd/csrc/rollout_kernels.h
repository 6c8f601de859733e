// rollout_kernels.h -- the fused roll-out's device code (arXiv 2408.00930,
// Sec. 2 and App. B: replicas step in place on the GPU, agents sample actions
// from a policy in device memory, roll-out data are stored in place).
//
// Templates over the environment kind: the library instantiates them for the
// built-in kinds (rollout.hip), and the user-kind composer compiles them at
// run time for an environment given as source (compose.cpp), so a user's
// environment runs in the same persistent kernel.
//
// Fused form: one persistent kernel runs the whole horizon. A workgroup owns a
// tile of R rows (env replicas, or the agents of whole market envs) and keeps
// their state in registers for all steps. The policy weights stay resident in
// VGPRs as MFMA A-operands (weight-stationary: wave w owns output features
// [w*H/NW, (w+1)*H/NW) of both hidden layers and a K-slice of the head);
// activations go through LDS as B-operands. Per step:
//   A  layer 1 (all waves)            -> h1 tile in LDS        | barrier
//   B  layer 2 (all waves)            -> own h2 slice in LDS   | wave-local
//   C  head partial over own K-slice  -> partials in LDS       | barrier
//   D  one thread per row: head = bias + sum of partials, sample, store the
//      record, step the dynamics, auto-reset, next observation -> LDS | barrier
#pragma once

#include <type_traits>

#include "device.h"
#include "envs.h"
#include "kernels.h"

namespace wsx {

// Entry sub + j G of a row's observation held on every lane of the row's G
// lanes, picked by selects (a branch per entry would split the step into
// many small blocks).
template <int OD, int G>
__device__ __forceinline__ float obs_entry(const float (&o)[OD], int j, int sub) {
    float v = 0.0f;
#pragma unroll
    for (int m = 0; m < G && j * G + m < OD; ++m) v = sub == m ? o[j * G + m] : v;
    return v;
}


static_assert(Reaction::NCACHE == kReactionCache, "one reaction cache size");

// ------------------------------------------------------ per-kind shapes --
template <class E>
struct HeadOf {
    static constexpr int NOUT = E::NACT ? E::NACT : 1;   // logits or one mean
    static constexpr int NH = NOUT + 1;                   // + value
    static constexpr int NHP = (NH + 15) / 16 * 16;
};

template <class E, int DT>
constexpr int kin_of() {
    return (E::OD + Mma<DT>::K - 1) / Mma<DT>::K * Mma<DT>::K;
}

// ------------------------------------------------------------ MLP tile --
__device__ __forceinline__ void wave_lds_sync() {
    // LDS writes of this wave complete before its later LDS reads of them.
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// HS selects how the head is spread over the waves. HS = 0 (split-K): wave w
// multiplies its own h2 features by its K-slice of the head for every head
// row, leaving NW partial sums per row (no extra barrier). HS = 1 (split-M):
// after a barrier, wave w computes head row tiles w, w + NW, ... over the whole
// K (one result per row; for wide heads whose partials would not fit in LDS);
// when the waves are a multiple of the head row tiles, the RS waves of one
// head row tile each take NT / RS of the row tiles instead.
// TRACE (a separate instantiation, used only by the policy-trace kernel): the
// quantised outputs of both hidden layers are also written to global memory,
// [row][H] codes of the policy format, so a checker can adopt the rounding
// decisions of the FP32 accumulation; the arithmetic is the same code.
template <int DT, int H, int NW, int NT, int KIN, int NHP, int HS, int OCC, bool TRACE = false>
struct Mlp {
    using M = Mma<DT>;
    using Frag = typename M::frag;
    static constexpr int K = M::K, KC = M::KC, EB = M::EB;
    static constexpr int FPW = H / NW;   // hidden features owned by a wave
    static constexpr int MT = FPW / 16;
    // FP8 products over K = 128 (layer 2; the head when a wave's K-slice, or
    // the split-M head's whole K, is a multiple of 128) take the 16x16x128
    // form, twice the matrix-core rate of the 16x16x32 one; layer 1 keeps
    // the narrow form (its K is the observation, padded to 32)
    using M2 = typename std::conditional<DT == DT_FP8 && H % 128 == 0, MmaF8K128, M>::type;
    using M3 = typename std::conditional<HS ? (DT == DT_FP8 && H % 128 == 0)
                                            : (DT == DT_FP8 && FPW % 128 == 0),
                                         MmaF8K128, M>::type;
    using Frag2 = typename M2::frag;
    using Frag3 = typename M3::frag;
    static constexpr int K2 = M2::K, KC2 = M2::KC, K3 = M3::K, KC3 = M3::KC;
    static constexpr int K1S = KIN / K, K2S = H / K2, K3S = FPW / K3, NHT = NHP / 16;
    static constexpr int NHW = HS ? (NHT + NW - 1) / NW : NHT;   // head tiles held by a wave
    static constexpr int KHS = HS ? H / K3 : K3S;                // head K-steps of a wave
    static constexpr int NPART = HS ? 1 : NW;                    // head results per row
    static constexpr int RS = (HS && NW % NHT == 0 && NT % (NW / NHT) == 0) ? NW / NHT : 1;
    static constexpr int NTR = NT / RS;                          // row tiles of a head job
    // the head row tile of a wave's job hw, and the first row tile of its job
    __device__ static int head_tile(int wave, int hw) {
        return HS ? (RS > 1 ? wave % NHT : wave + hw * NW) : hw;
    }
    __device__ static int head_row0(int wave) { return RS > 1 ? (wave / NHT) * NTR : 0; }
    static constexpr int R = 16 * NT;
    static constexpr int P_IN = KIN * EB + 16;   // LDS row pitches (bytes)
    static constexpr int P_H = H * EB + 16;
    static constexpr int P_PART = NHP + 4;       // floats
    static constexpr int OFF_IN = 0;
    static constexpr int OFF_H1 = OFF_IN + R * P_IN;
    static constexpr int OFF_H2 = OFF_H1 + R * P_H;   // split-M only
    // split-M writes the head after a barrier that follows the last read of
    // h1, so its results reuse the h1 tile; split-K takes each wave's h2
    // features from its registers (no h2 tile) and writes partials there
    static constexpr int OFF_PART = HS ? OFF_H1 : OFF_H2;
    // per-feature accumulator start (bias / output scale) and tanh factor
    // (2 log2 e * output scale) of both hidden layers: [4][H] floats
    static constexpr int OFF_TAB = HS ? OFF_H2 + R * P_H : OFF_PART + NPART * R * P_PART * 4;
    static constexpr int WPS = (NW / 4 > OCC ? NW / 4 : OCC);   // waves per SIMD
    // Four-wave kernels sharing a SIMD with another workgroup keep W1 in LDS
    // (read per step, so its registers are free outside layer 1): [wave][mt]
    // [ks][lane] fragments, each lane reading its own 16 (8, 4) bytes.
    static constexpr bool W1_LDS = NW == 4 && WPS >= 2;
    static constexpr int OFF_W1 = OFF_TAB + 4 * H * 4;
    static constexpr int W1_BYTES = W1_LDS ? NW * MT * K1S * 64 * (int)sizeof(Frag) : 0;
    // the same for the head weights of the split-K head ([wave][hw][ks][lane])
    static constexpr bool W3_LDS = W1_LDS && !HS;
    static constexpr int OFF_W3 = OFF_W1 + W1_BYTES;
    static constexpr int W3_BYTES = W3_LDS ? NW * NHW * KHS * 64 * (int)sizeof(Frag3) : 0;
    static constexpr int BYTES = OFF_W3 + W3_BYTES;
    static_assert(!HS || P_PART * 4 <= P_H, "head results fit in the h1 tile");
    static_assert(FPW % 16 == 0 && (HS || FPW % K3 == 0) && KIN % K == 0 && H % K2 == 0 && H % K3 == 0,
                  "tile shape");
    static_assert(BYTES <= 160 * 1024, "LDS budget");

    static constexpr int DTYPE = DT;
    // software pipelining of the dense layers (see dense_tanh): with at most
    // two waves per SIMD and at most 64 registers of layer-2 weights per lane,
    // or with one wave per SIMD and at most four output tiles per wave
    static constexpr int W2_REGS = MT * K2S * (int)sizeof(Frag2) / 4;
    static constexpr bool PIPE_ON =
        (WPS <= 2 && W2_REGS <= 64) || (WPS == 1 && MT <= 4);

    Frag w1[MT][K1S];
    Frag2 w2[MT][K2S];
    Frag3 w3[NHW][KHS];
    float o3[NHW][4];                  // head output scale
    float inv_q1, inv_q2;              // 1 / scale of the h1 and h2 quantisation
    char* tr_act[2];                   // TRACE: the tile's first row of each layer's codes
    int tr_rows;                       // TRACE: valid rows of the tile

    __device__ static Frag& w1_lds(char* base, int wave, int mt, int ks, int lane) {
        return reinterpret_cast<Frag*>(base)[((wave * MT + mt) * K1S + ks) * 64 + lane];
    }
    __device__ static Frag3& w3_lds(char* base, int wave, int hw, int ks, int lane) {
        return reinterpret_cast<Frag3*>(base)[((wave * NHW + hw) * KHS + ks) * 64 + lane];
    }

    __device__ static float row_scale(const float* s, int m, int m_valid) {
        return (s != nullptr && m < m_valid) ? s[m] : 1.0f;
    }

    // Weights into registers and the per-feature table into LDS (the caller
    // synchronises the workgroup before the first forward).
    __device__ void load(const PolicyArgs& p, char* smem, int wave, int lane, int tid) {
        const int lr = lane & 15, kq = (lane >> 4) * KC;
        const float a0 = DT == DT_FP8 ? p.act_scale[0] : 1.0f;
        const float a1 = DT == DT_FP8 ? p.act_scale[1] : 1.0f;
        const float a2 = DT == DT_FP8 ? p.act_scale[2] : 1.0f;
        inv_q1 = 1.0f / a1;
        inv_q2 = 1.0f / a2;
        float* tab = reinterpret_cast<float*>(smem + OFF_TAB);
        for (int m = tid; m < H; m += NW * 64) {
            const float sc1 = row_scale(p.s1, m, H) * a0;
            const float sc2 = row_scale(p.s2, m, H) * a1;
            tab[m] = p.b1[m] / sc1;
            tab[H + m] = kTwoLog2e * sc1;
            tab[2 * H + m] = p.b2[m] / sc2;
            tab[3 * H + m] = kTwoLog2e * sc2;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int m = wave * FPW + mt * 16 + lr;
#pragma unroll
            for (int ks = 0; ks < K1S; ++ks) {
                load_a(w1[mt][ks], p.w1, p.d_in, m, H, ks * K + kq, p.d_in);
                if constexpr (W1_LDS)
                    w1_lds(reinterpret_cast<char*>(tab) + (OFF_W1 - OFF_TAB), wave, mt, ks, lane) =
                        w1[mt][ks];
            }
#pragma unroll
            for (int ks = 0; ks < K2S; ++ks)
                load_a(w2[mt][ks], p.w2, H, m, H, ks * K2 + (lane >> 4) * KC2, H);
        }
#pragma unroll
        for (int hw = 0; hw < NHW; ++hw) {
            const int ht = head_tile(wave, hw);   // head row tile
            const int m = ht * 16 + lr;
#pragma unroll
            for (int ks = 0; ks < KHS; ++ks) {
                if constexpr (HS) {
                    load_a(w3[hw][ks], p.w3, H, m, p.n_head, ks * K3 + (lane >> 4) * KC3, H);
                } else {
                    // K element e of lane group q is this wave's layer-2 output
                    // (tile mt, accumulator row i): idx = ks KC3 + e, mt = idx / 4
                    const int q = lane >> 4;
                    load_a_cols(w3[hw][ks], p.w3, H, m, p.n_head, [&](int e) {
                        const int idx = ks * KC3 + e;
                        return wave * FPW + (idx >> 2) * 16 + 4 * q + (idx & 3);
                    });
                    if constexpr (W3_LDS)
                        w3_lds(reinterpret_cast<char*>(tab) + (OFF_W3 - OFF_TAB), wave, hw, ks,
                               lane) = w3[hw][ks];
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) o3[hw][i] = row_scale(p.s3, ht * 16 + 4 * (lane >> 4) + i, p.n_head) * a2;
        }
    }

    // Accumulators of this wave's MT output tiles for row tile `nt`: the
    // per-feature start `ini` plus W times the row tile's inputs.
    template <class MM, int KS>
    __device__ __forceinline__ static void mma_rows(f32x4 (&acc)[MT],
                                                    const typename MM::frag (&w)[MT][KS],
                                                    const float4 (&ini)[MT], const char* in,
                                                    int p_in, int nt, int lane) {
        const int lr = lane & 15, kq = (lane >> 4) * MM::KC;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{ini[mt].x, ini[mt].y, ini[mt].z, ini[mt].w};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const typename MM::frag b = MM::lds(in + (nt * 16 + lr) * p_in + (ks * MM::K + kq) * EB);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = MM::mma(w[mt][ks], b, acc[mt]);
        }
    }

    // Layer outputs of one accumulator tile, quantised for the next product:
    // four BF16 (uint2), four FP8 codes (uint32) or four floats.
    typedef typename std::conditional<
        DT == DT_BF16, uint2, typename std::conditional<DT == DT_FP8, uint32_t, float4>::type>::type
        Packed;

    __device__ __forceinline__ static Packed tanh_pack(const f32x4& a, const float4& k, float q) {
        if constexpr (DT == DT_FP8) {
            return pack_fp8x4(tanh_scaled_q(a[0], k.x, q), tanh_scaled_q(a[1], k.y, q),
                              tanh_scaled_q(a[2], k.z, q), tanh_scaled_q(a[3], k.w, q));
        } else if constexpr (DT == DT_BF16) {
            return make_uint2(pack_bf16x2(tanh_scaled(a[0], k.x), tanh_scaled(a[1], k.y)),
                              pack_bf16x2(tanh_scaled(a[2], k.z), tanh_scaled(a[3], k.w)));
        } else {
            return make_float4(tanh_scaled(a[0], k.x), tanh_scaled(a[1], k.y),
                               tanh_scaled(a[2], k.z), tanh_scaled(a[3], k.w));
        }
    }

    // B fragment of head K-step ks from this wave's packed layer-2 outputs of
    // one row tile (the order load() gave the head weights).
    __device__ __forceinline__ static Frag3 head_frag(const Packed (&pk)[MT], int ks) {
        if constexpr (DT == DT_BF16) {
            const uint4 u = make_uint4(pk[2 * ks].x, pk[2 * ks].y, pk[2 * ks + 1].x, pk[2 * ks + 1].y);
            return __builtin_bit_cast(Frag3, u);
        } else if constexpr (std::is_same<M3, MmaF8K128>::value) {
            // 32 elements: the packed outputs of tiles 8 ks .. 8 ks + 7
            Frag3 f;
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = (int)pk[8 * ks + i];
            return f;
        } else if constexpr (DT == DT_FP8) {
            return (long)((uint64_t)pk[2 * ks] | ((uint64_t)pk[2 * ks + 1] << 32));
        } else {
            const float4 v = pk[ks >> 2];
            const int i = ks & 3;
            return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
        }
    }

    // tanh of row tile `nt`'s accumulators: quantised into `out` ([R][H]) for
    // the next layer (layer 1, split-M layer 2), or fed to the split-K head
    // MFMAs of this row tile (HEAD: layer 2 of a split-K head).
    template <bool HEAD, int LAYER>
    __device__ __forceinline__ void tanh_rows(const f32x4 (&acc)[MT], const float4 (&kx)[MT],
                                              char* out, float q, int nt, int wave, int lane,
                                              f32x4 (&acc3)[NHW][NT]) {
        const int lr = lane & 15;
        Packed pk[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) pk[mt] = tanh_pack(acc[mt], kx[mt], DT == DT_FP8 ? q : 1.0f);
        if constexpr (TRACE) {
            if (nt * 16 + lr < tr_rows) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int feat = wave * FPW + mt * 16 + 4 * (lane >> 4);
                    *reinterpret_cast<Packed*>(tr_act[LAYER] +
                                               ((size_t)(nt * 16 + lr) * H + feat) * EB) = pk[mt];
                }
            }
        }
        if constexpr (HEAD) {
#pragma unroll
            for (int ks = 0; ks < KHS; ++ks) {
                const Frag3 b = head_frag(pk, ks);
#pragma unroll
                for (int hw = 0; hw < NHW; ++hw) acc3[hw][nt] = M3::mma(w3[hw][ks], b, acc3[hw][nt]);
            }
        } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int feat = wave * FPW + mt * 16 + 4 * (lane >> 4);
                *reinterpret_cast<Packed*>(out + (nt * 16 + lr) * P_H + feat * EB) = pk[mt];
            }
        }
    }

    // Dense layer of this wave's MT output tiles for all NT row tiles, then
    // tanh and quantisation (into `out`, or into the split-K head's MFMAs
    // with HEAD). With PIPE_ON the loop is software-pipelined over row tiles:
    // the MFMAs of row tile n + 1 are issued ahead of the tanh of row tile n,
    // so the matrix core and the vector ALU of the SIMD work at the same time
    // (this holds two tiles of accumulators and the next tile's operands in
    // registers; without it -- kernels with four or more waves per SIMD, or
    // whose layer-2 weights take more than 64 registers per lane -- each row
    // tile is multiplied, then activated). `tab` holds the layer's
    // accumulator starts and tanh factors.
    template <class MM, int KS, bool HEAD, int LAYER>
    __device__ __forceinline__ void dense_tanh(const typename MM::frag (&w)[MT][KS], const float* tab,
                                               const char* in, int p_in, char* out, float inv_q,
                                               int wave, int lane, f32x4 (&acc3)[NHW][NT]) {
        float4 ini[MT], kx[MT];
        auto per_feature = [&]() {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int feat = wave * FPW + mt * 16 + 4 * (lane >> 4);
                ini[mt] = *reinterpret_cast<const float4*>(tab + feat);
                if constexpr (DT == DT_FP8)
                    kx[mt] = *reinterpret_cast<const float4*>(tab + H + feat);
                else
                    kx[mt] = make_float4(kTwoLog2e, kTwoLog2e, kTwoLog2e, kTwoLog2e);
            }
        };
        if constexpr (!PIPE_ON) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                f32x4 acc[MT];
                per_feature();   // re-read per row tile: fewer live registers
                mma_rows<MM, KS>(acc, w, ini, in, p_in, nt, lane);
                tanh_rows<HEAD, LAYER>(acc, kx, out, inv_q, nt, wave, lane, acc3);
            }
            return;
        }
        per_feature();
        f32x4 acc[2][MT];
        mma_rows<MM, KS>(acc[0], w, ini, in, p_in, 0, lane);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (nt + 1 < NT) mma_rows<MM, KS>(acc[(nt + 1) & 1], w, ini, in, p_in, nt + 1, lane);
            tanh_rows<HEAD, LAYER>(acc[nt & 1], kx, out, inv_q, nt, wave, lane, acc3);
            if (nt + 1 < NT) {
                // all LDS reads of the next row tile first, a few vector
                // instructions while they land, then one MFMA at a time, each
                // followed by a share of the tanh's vector work
                constexpr int NM = MT * KS + (HEAD ? NHW * KHS : 0);
                constexpr int NVT = MT * 4 * 6, NV0 = 8;
                constexpr int NV = (NVT - NV0 + NM - 1) / NM;
                __builtin_amdgcn_sched_group_barrier(0x100, KS, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, NV0, 0);
#pragma unroll
                for (int i = 0; i < NM; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);
                }
                __builtin_amdgcn_sched_barrier(0);   // one scheduling region per row tile
            }
        }
    }

    // Phases A-C. The caller synchronises the workgroup afterwards.
    __device__ void forward(char* smem, int wave, int lane) {
        const float* tab = reinterpret_cast<const float*>(smem + OFF_TAB);
        const int lr = lane & 15, kq = (lane >> 4) * KC;
        f32x4 acc[NHW][NT];
#pragma unroll
        for (int hw = 0; hw < NHW; ++hw)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[hw][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (W1_LDS) {
            Frag w1r[MT][K1S];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int ks = 0; ks < K1S; ++ks) w1r[mt][ks] = w1_lds(smem + OFF_W1, wave, mt, ks, lane);
            dense_tanh<M, K1S, false, 0>(w1r, tab, smem + OFF_IN, P_IN, smem + OFF_H1, inv_q1, wave,
                                         lane, acc);
        } else {
            dense_tanh<M, K1S, false, 0>(w1, tab, smem + OFF_IN, P_IN, smem + OFF_H1, inv_q1, wave,
                                         lane, acc);
        }
        __syncthreads();
        if constexpr (!HS) {
            if constexpr (W3_LDS) {   // head weights back from LDS for this step
#pragma unroll
                for (int hw = 0; hw < NHW; ++hw)
#pragma unroll
                    for (int ks = 0; ks < KHS; ++ks) w3[hw][ks] = w3_lds(smem + OFF_W3, wave, hw, ks, lane);
            }
            // split-K: the head consumes each wave's own h2 from its registers
            dense_tanh<M2, K2S, true, 1>(w2, tab + 2 * H, smem + OFF_H1, P_H, nullptr, inv_q2, wave,
                                         lane, acc);
        } else {
            dense_tanh<M2, K2S, false, 1>(w2, tab + 2 * H, smem + OFF_H1, P_H, smem + OFF_H2, inv_q2,
                                          wave, lane, acc);
            __syncthreads();   // every wave reads all of h2
            const char* h2 = smem + OFF_H2 + head_row0(wave) * 16 * P_H;
            const int kq3 = (lane >> 4) * KC3;
#pragma unroll
            for (int ks = 0; ks < KHS; ++ks) {
                Frag3 b[NTR];
#pragma unroll
                for (int i = 0; i < NTR; ++i)
                    b[i] = M3::lds(h2 + (i * 16 + lr) * P_H + (ks * K3 + kq3) * EB);
#pragma unroll
                for (int hw = 0; hw < NHW; ++hw) {
                    if (head_tile(wave, hw) >= NHT) break;
#pragma unroll
                    for (int i = 0; i < NTR; ++i) acc[hw][i] = M3::mma(w3[hw][ks], b[i], acc[hw][i]);
                }
            }
        }
        float* part = reinterpret_cast<float*>(smem + OFF_PART) + (HS ? 0 : wave * R * P_PART) +
                      (HS ? head_row0(wave) * 16 * P_PART : 0);
#pragma unroll
        for (int hw = 0; hw < NHW; ++hw) {
            const int ht = head_tile(wave, hw);
            if (HS && ht >= NHT) break;
#pragma unroll
            for (int i = 0; i < (HS ? NTR : NT); ++i) {
                const f32x4 a = acc[hw][i];
                const int j = ht * 16 + 4 * (lane >> 4);
                *reinterpret_cast<float4*>(part + (i * 16 + lr) * P_PART + j) =
                    make_float4(a[0] * o3[hw][0], a[1] * o3[hw][1], a[2] * o3[hw][2], a[3] * o3[hw][3]);
            }
        }
    }

    // Head outputs of tile row r: bias + partials summed in wave order (split-K)
    // or bias + the one result (split-M).
    template <int NH>
    __device__ static void head_row(const char* smem, const float* b3, int r, float (&h)[NH]) {
        const float* part = reinterpret_cast<const float*>(smem + OFF_PART);
#pragma unroll
        for (int j = 0; j < NH; ++j) h[j] = 0.0f;
#pragma unroll
        for (int w = 0; w < NPART; ++w) {
            const float* pr = part + (w * R + r) * P_PART;
#pragma unroll
            for (int j4 = 0; j4 < NHP / 4; ++j4) {
                if (j4 * 4 >= NH) break;
                const float4 v = *reinterpret_cast<const float4*>(pr + j4 * 4);
                if (j4 * 4 + 0 < NH) h[j4 * 4 + 0] += v.x;
                if (j4 * 4 + 1 < NH) h[j4 * 4 + 1] += v.y;
                if (j4 * 4 + 2 < NH) h[j4 * 4 + 2] += v.z;
                if (j4 * 4 + 3 < NH) h[j4 * 4 + 3] += v.w;
            }
        }
#pragma unroll
        for (int j = 0; j < NH; ++j) h[j] += b3[j];
    }

    // Head outputs [j0, j0 + C) (those below NH - 1) and the value output
    // (index NH - 1) of tile row r, summed in the same order as head_row.
    template <int NH, int C>
    __device__ static void head_block(const char* smem, const float (&b3b)[C], float b3v, int r,
                                      int j0, float (&hb)[C], float& hv) {
        const float* part = reinterpret_cast<const float*>(smem + OFF_PART);
        float acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0f;
        float accv = 0.0f;
#pragma unroll
        for (int w = 0; w < NPART; ++w) {
            const float* pr = part + (w * R + r) * P_PART;
#pragma unroll
            for (int c = 0; c < C; ++c) {   // entries past the logits read the value and add 0
                const int j = j0 + c < NH - 1 ? j0 + c : NH - 1;
                const float v = pr[j];
                acc[c] += j0 + c < NH - 1 ? v : 0.0f;
            }
            accv += pr[NH - 1];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) hb[c] = acc[c] + b3b[c];
        hv = accv + b3v;
    }

    // Quantised observation row into the input tile; lane `sub` of the row's
    // G lanes writes the elements congruent to sub mod G.
    template <int OD, int G>
    __device__ static void put_obs(char* smem, int r, const float (&o)[OD], float inv_q0, int sub) {
        char* p = smem + OFF_IN + r * P_IN;
#pragma unroll
        for (int j = 0; j < (OD + G - 1) / G; ++j) {
            const float v = obs_entry<OD, G>(o, j, sub);
            if (j * G + G <= OD || sub + j * G < OD) store1<DT>(p + (sub + j * G) * EB, v, inv_q0);
        }
    }
    // The same from a lane's slice: entries k = sub + j G of the row.
    template <int OD, int G>
    __device__ static void put_obs_slice(char* smem, int r, const float* o, float inv_q0, int sub) {
        char* p = smem + OFF_IN + r * P_IN;
#pragma unroll
        for (int j = 0; j < (OD + G - 1) / G; ++j)
            if (OD % G == 0 || sub + j * G < OD) store1<DT>(p + (sub + j * G) * EB, o[j], inv_q0);
    }
};

// ------------------------------------------------------------- sampling --
// The head block of a row's lane: lane `sub` of G holds logits
// [sub * C, sub * C + C) of a categorical head; a Gaussian head's mean is on
// every lane.
template <class E, int G>
struct Block {
    static constexpr int C = E::NACT ? (E::NACT + G - 1) / G : 1;
    __device__ static int first(int sub) { return E::NACT ? sub * C : 0; }
};

// Categorical draw over the row's G lanes: softmax with the maximum
// subtracted, CDF in index order, a = min{k : u < C_k} (K - 1 if none).
// Every lane returns the same action and log-probability.
template <int K, int G, int C>
__device__ __forceinline__ int sample_categorical(const float (&lg)[C], int sub, float u,
                                                  float& logp) {
    const int j0 = sub * C;
    float mx = -__builtin_inff();
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (j0 + c < K) mx = fmaxf(mx, lg[c]);
    mx = group_max<G>(mx);
    float e[C];
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {   // exp of every entry, then a select: no branch
        // exp_nonpos measured faster for rows of one and four lanes (CartPole
        // 0.438 -> 0.424 ms, market 9.88 -> 9.78 ms) but slower for the
        // reaction's 16-lane rows (3.12 -> 3.24 ms, same box), which keep expf
        const float ex = G <= 4 ? exp_nonpos(lg[c] - mx) : expf(lg[c] - mx);
        e[c] = j0 + c < K ? ex : 0.0f;
        s += e[c];
    }
    const float z = group_sum<G>(s);
    const float uz = u * z;   // u < C_k tested as u z < (unnormalised) C_k: no division
    float acc = group_prefix<G>(s, sub);
    int cand = K;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        acc += e[c];
        if (cand == K && j0 + c < K && uz < acc) cand = j0 + c;
    }
    int a = group_min<G>(cand);
    if (a >= K) a = K - 1;
    float la = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (j0 + c == a) la = lg[c];
    la = group_sum<G>(la);   // only the owner contributes
    logp = (la - mx) - log_hw(z);   // z >= 1 (its largest term is 1)
    return a;
}

template <class E>
struct Act {
    int index;
    float value;
};

// The part of a draw that does not depend on the policy's outputs: the
// categorical uniform, or the Gaussian's standard normal and log-probability.
// The fused kernel computes it for step t + 1 beside the dynamics of step t.
template <class E>
struct Pre {
    float u;      // categorical: the uniform; Gaussian: z
    float logp;   // Gaussian: log-probability of z
};

template <class E>
__device__ __forceinline__ Pre<E> prepare(const RngKey& key, uint32_t t, uint32_t row,
                                          float log_std) {
    const Words w = draw(key, t, row, PURPOSE_ACTION, 0);
    Pre<E> p{0.0f, 0.0f};
    if constexpr (E::NACT > 0) {
        p.u = unit_uniform(w.w[0]);
    } else {
        float zc, zs;
        gauss_pair(unit_uniform(w.w[0]), unit_uniform(w.w[1]), zc, zs);
        p.u = zc;
        p.logp = -0.5f * zc * zc - log_std - 0.91893853320467274f;   // log(2 pi) / 2
    }
    return p;
}

// The action from the head block and the prepared draw.
template <class E, int G, int C>
__device__ __forceinline__ Act<E> decide(const float (&hb)[C], int sub, const Pre<E>& p,
                                         float sigma, float& logp) {
    Act<E> act{0, 0.0f};
    if constexpr (E::NACT > 0) {
        act.index = sample_categorical<E::NACT, G, C>(hb, sub, p.u, logp);
        act.value = (float)act.index;
    } else {
        act.value = hb[0] + sigma * p.u;
        logp = p.logp;
    }
    return act;
}

// Draw the action of row `row` at step t from its head block.
template <class E, int G, int C>
__device__ __forceinline__ Act<E> choose(const float (&hb)[C], int sub, const RngKey& key,
                                         uint32_t t, uint32_t row, float log_std, float& logp) {
    return decide<E, G, C>(hb, sub, prepare<E>(key, t, row, log_std), expf(log_std), logp);
}

// ------------------------------------------------- global-memory views --
// The fused kernels read their segment's pointers from LDS, so the compiler
// cannot tell that they point to global memory and would use flat
// instructions, which count against the LDS counter too: every later LDS wait
// and barrier would wait for the step's record stores to reach memory. The
// view carries the record pointers as global (address space 1) ones.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

struct GTraj {
    gptr<float> obs;
    gptr<void> action;
    gptr<float> reward;
    gptr<uint8_t> done;
    gptr<float> value, logp, last_value;
};

__device__ __forceinline__ GTraj global_view(const TrajArgs& t) {
    return GTraj{(gptr<float>)t.obs,    (gptr<void>)t.action, (gptr<float>)t.reward,
                 (gptr<uint8_t>)t.done, (gptr<float>)t.value, (gptr<float>)t.logp,
                 (gptr<float>)t.last_value};
}

template <class E>
__device__ __forceinline__ void store_action(const GTraj& tr, size_t idx, const Act<E>& a) {
    if constexpr (E::NACT > 0)
        ((gptr<uint8_t>)tr.action)[idx] = (uint8_t)a.index;
    else
        ((gptr<float>)tr.action)[idx] = a.value;
}

template <class E>
__device__ __forceinline__ void store_action(const TrajArgs& tr, size_t idx, const Act<E>& a) {
    if constexpr (E::NACT > 0)
        static_cast<uint8_t*>(tr.action)[idx] = (uint8_t)a.index;
    else
        static_cast<float*>(tr.action)[idx] = a.value;
}

template <class E>
__device__ __forceinline__ Act<E> load_action(const TrajArgs& tr, size_t idx) {
    Act<E> a{0, 0.0f};
    if constexpr (E::NACT > 0)
        a.index = static_cast<const uint8_t*>(tr.action)[idx];
    else
        a.value = static_cast<const float*>(tr.action)[idx];
    return a;
}

// ------------------------------------------------------------- env glue --
template <class E>
__device__ __forceinline__ void load_state(const EnvArgs& env, int64_t row, float (&s)[E::SR]) {
#pragma unroll
    for (int i = 0; i < E::SD; ++i) s[i] = env.state[(size_t)i * env.n_rows + row];
    E::complete(s);   // derived register-state entries (sin / cos of the angles)
}

template <class E, int G>
__device__ __forceinline__ void save_state(const EnvArgs& env, int64_t row, const float (&s)[E::SR],
                                           int sub) {
#pragma unroll
    for (int i = 0; i < E::SD; ++i)
        if (i % G == sub) env.state[(size_t)i * env.n_rows + row] = s[i];
}

// Lane `sub` of the row's G lanes stores entries k = sub + j G (obs_entry
// picks them by selects).
template <int OD, int G, class P>
__device__ __forceinline__ void store_obs(P dst, const float (&o)[OD], int sub) {
#pragma unroll
    for (int j = 0; j < (OD + G - 1) / G; ++j) {
        const float v = obs_entry<OD, G>(o, j, sub);
        if (j * G + G <= OD || sub + j * G < OD) dst[sub + j * G] = v;
    }
}

// State and observation slices: lane `sub` of a row's group of G holds the
// entries i = sub + j G (the market's state is its observation, and every
// entry evolves on its own, so no lane needs the others').
template <class E, int G>
__device__ __forceinline__ void load_slice(const EnvArgs& env, int64_t row, float (&s)[E::SD / G],
                                           int sub) {
#pragma unroll
    for (int j = 0; j < E::SD / G; ++j) s[j] = env.state[(size_t)(sub + j * G) * env.n_rows + row];
}
template <class E, int G>
__device__ __forceinline__ void save_slice(const EnvArgs& env, int64_t row,
                                           const float (&s)[E::SD / G], int sub) {
#pragma unroll
    for (int j = 0; j < E::SD / G; ++j) env.state[(size_t)(sub + j * G) * env.n_rows + row] = s[j];
}
template <int OD, int G, class P>
__device__ __forceinline__ void store_obs_slice(P dst, const float* o, int sub) {
#pragma unroll
    for (int j = 0; j < (OD + G - 1) / G; ++j)
        if (OD % G == 0 || sub + j * G < OD) dst[sub + j * G] = o[j];
}

// The reaction walk's slice of a row on lane `sub`: coordinates x[sub + m G]
// (zero past the last), then the energy (on every lane).
template <int G>
__device__ __forceinline__ void load_rx_slice(const EnvArgs& env, int64_t row, float* s, int sub) {
    constexpr int NX = (Reaction::NDIM + G - 1) / G;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
        const int i = sub + m * G;
        s[m] = i < Reaction::NDIM ? env.state[(size_t)i * env.n_rows + row] : 0.0f;
    }
    s[NX] = env.state[(size_t)Reaction::NDIM * env.n_rows + row];
}
template <int G>
__device__ __forceinline__ void save_rx_slice(const EnvArgs& env, int64_t row, const float* s,
                                              int sub) {
    constexpr int NX = (Reaction::NDIM + G - 1) / G;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
        const int i = sub + m * G;
        if (i < Reaction::NDIM) env.state[(size_t)i * env.n_rows + row] = s[m];
    }
    if (sub == Reaction::NDIM % G) env.state[(size_t)Reaction::NDIM * env.n_rows + row] = s[NX];
}

// Stage the reaction potential in LDS: A, centres, -log2(e)/(2 w^2) (so a
// well's term is amp * 2^(d * that), one v_exp_f32), amplitudes.
__device__ __forceinline__ void stage_params(float* dst, const float* src, int tid, int nthreads) {
    constexpr int NA = Reaction::NDIM * Reaction::NDIM + Reaction::NG * Reaction::NDIM;
    for (int i = tid; i < Reaction::PARAM_FLOATS; i += nthreads) {
        float v = src[i];
        if (i >= NA && i < NA + Reaction::NG) v = -0.72134752044448170f / (v * v);   // log2(e) / 2
        dst[i] = v;
    }
}

// The reaction's LDS: the potential block, then the cache of the tile's rows,
// row-major with an odd pitch of doubles so that the lanes of a row (entries
// sub + m G) and the rows of a wave fall on different banks.
constexpr int kRxCacheOff = (Reaction::PARAM_FLOATS * 4 + 15) / 16 * 16;
constexpr int kRxCachePitch = Reaction::NCACHE + 1;

template <class E>
constexpr int extra_lds_bytes(int R) {
    if constexpr (E::KIND == Reaction::KIND) return kRxCacheOff + kRxCachePitch * R * 8;
    if constexpr (E::KIND == Market::KIND) return 2 * R * 2 * 4;   // [parity][slot][D, S]
    return 0;
}

__device__ __forceinline__ uint32_t step_base(const EnvArgs& env) {
    return env.step_ptr ? env.step_ptr[0] + env.t0 : env.t0;
}

// The random-stream key of a launch; a graph-captured launch reads the reset
// epoch from the device copy beside the step counter, so one captured graph
// serves every epoch.
__device__ __forceinline__ RngKey rng_key(const EnvArgs& env) {
    return RngKey{env.k0, env.k1, env.step_ptr ? env.step_ptr[1] : env.epoch};
}

__device__ __forceinline__ Tile tile_of(const EnvArgs& env, int tile) {
    if (env.tiles) return env.tiles[tile];
    const int rows = env.tile_rows;   // <= the kernel's row capacity
    Tile t;
    t.row0 = tile * rows;
    t.row1 = (int)min((int64_t)(tile + 1) * rows, env.n_rows);
    t.env0 = t.row0;
    t.env1 = t.row1;
    return t;
}

// Global row of tile entry i (row0 <= i < row1): the market's tiles list their
// rows in the row map, the other kinds' tiles are row ranges.
__device__ __forceinline__ int tile_row(const EnvArgs& env, int i) {
    return env.row_map ? env.row_map[i] : i;
}

// ---------------------------------------------------------- fused form --
// The launch covers the tiles of one or more segments (roll-out requests that
// share the policy): tile b of the launch belongs to the segment whose
// tile_begin is the largest one <= b.
// A copy of a wave-uniform struct in scalar registers (every dword through
// v_readfirstlane).
template <class T>
__device__ __forceinline__ T uniform(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "whole dwords");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// Index of the segment that tile `tile` of the launch belongs to.
__device__ __forceinline__ int segment_index(const Batch& b, int tile) {
    if (!b.table) {
        int i = 0;
        while (i + 1 < b.n_segs && b.inl[i + 1].tile_begin <= tile) ++i;
        return i;
    }
    int lo = 0, hi = b.n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.table[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Copy segment i into LDS (`dst`), one dword per thread. The inline segments
// are read through the kernel-argument segment pointer (the Batch is the
// kernel's only argument, at offset 0): indexing the argument itself would
// make the compiler copy all of it to scratch. The caller synchronises.
__device__ __forceinline__ void stage_segment(const Batch& b, int i, Segment* dst, int tid,
                                              int nthreads) {
    typedef const __attribute__((address_space(4))) uint32_t KArgWord;
    constexpr int NW32 = (int)(sizeof(Segment) / 4);
    static_assert(sizeof(Segment) % 4 == 0, "segment of whole dwords");
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    if (b.table) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(b.table + i);
        for (int k = tid; k < NW32; k += nthreads) d[k] = src[k];
    } else {
        KArgWord* src = (KArgWord*)((const __attribute__((address_space(4))) char*)
                                        __builtin_amdgcn_kernarg_segment_ptr() +
                                    __builtin_offsetof(Batch, inl) + (size_t)i * sizeof(Segment));
        for (int k = tid; k < NW32; k += nthreads) d[k] = src[k];
    }
}

// Returns and GAE of a tile's rows after its steps, FP64 (the recursions of
// the returns kernels): thread tid takes row tid % n of the tile's n rows and
// time segment tid / n of the horizon. Each segment composes its steps' affine
// maps backwards (x -> b + c x, for G and for A), the compositions meet in
// `buf` (LDS, 32 bytes per row and segment), and each segment then reruns its
// recursion from the carry of the later segments and writes its outputs. A
// segment's records are loaded GB steps at a time with every load in flight
// (one chain of dependent loads per step would cost a memory round trip
// each), and kept in registers for the second pass when the segment is one
// block. The records are the workgroup's own stores, visible after the
// barrier that precedes the call; `buf` is reused by the caller afterwards.
template <int NTHR, int GB>
__device__ void tile_gae(const EnvArgs& env, const GTraj& tr, const GaeArgs& g, const Tile& tl,
                         int horizon, double* buf, int buf_bytes, int tid) {
    const int n = tl.row1 - tl.row0;
    if (n <= 0 || horizon <= 0) return;
    int nseg = min(min(NTHR / n, buf_bytes / (32 * n)), horizon);
    const int len = (horizon + nseg - 1) / nseg;
    nseg = (horizon + len - 1) / len;   // every segment non-empty
    const int r = tid % n, q = tid / n;
    const bool live = q < nseg;
    const size_t rows = (size_t)env.n_rows;
    const int row = live ? tile_row(env, tl.row0 + r) : 0;
    const int lo = q * len, hi = min(horizon, lo + len);
    const double gam = g.gamma, gl = g.gamma * g.lambda;
    const double v_end = (live && g.bootstrap) ? (double)tr.last_value[row] : 0.0;
    const double v_hi = !live ? 0.0 : hi == horizon ? v_end : (double)tr.value[(size_t)hi * rows + row];
    double* mine = buf + ((size_t)q * n + r) * 4;
    float br[GB], bv[GB], bk[GB];   // a block of records
    // steps tb - 1, tb - 2, ..., down to max(lo, tb - GB)
    auto load_block = [&](int tb) {
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            const int t = tb - 1 - u;
            const size_t i = (size_t)(t >= lo ? t : lo) * rows + row;
            br[u] = tr.reward[i];
            bv[u] = tr.value[i];
            bk[u] = tr.done[i] ? 0.0f : 1.0f;
        }
    };
    if (live) {
        double cg = 1.0, bg = 0.0, ca = 1.0, ba = 0.0, v_next = v_hi;
        for (int tb = hi; tb > lo; tb -= GB) {
            load_block(tb);
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                if (tb - 1 - u >= lo) {
                    const double rw = br[u], v = bv[u], keep = bk[u];
                    const double c = gam * keep, e = gl * keep;
                    const double delta = rw + c * v_next - v;
                    bg = rw + c * bg;
                    cg = c * cg;
                    ba = delta + e * ba;
                    ca = e * ca;
                    v_next = v;
                }
            }
        }
        mine[0] = cg;
        mine[1] = bg;
        mine[2] = ca;
        mine[3] = ba;
    }
    __syncthreads();
    if (live) {
        double G = v_end, A = 0.0;
        for (int p = nseg - 1; p > q; --p) {
            const double* m = buf + ((size_t)p * n + r) * 4;
            G = m[1] + m[0] * G;
            A = m[3] + m[2] * A;
        }
        double v_next = v_hi;
        const bool kept = hi - lo <= GB;   // the one block is still in registers
        for (int tb = hi; tb > lo; tb -= GB) {
            if (!kept) load_block(tb);
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const int t = tb - 1 - u;
                if (t >= lo) {
                    const double rw = br[u], v = bv[u], keep = bk[u];
                    const double c = gam * keep, e = gl * keep;
                    const double delta = rw + c * v_next - v;
                    G = rw + c * G;
                    A = delta + e * A;
                    v_next = v;
                    const size_t i = (size_t)t * rows + row;
                    if (g.out_f64) {
                        ((gptr<double>)g.ret)[i] = G;
                        ((gptr<double>)g.adv)[i] = A;
                    } else {
                        ((gptr<float>)g.ret)[i] = (float)G;
                        ((gptr<float>)g.adv)[i] = (float)A;
                    }
                }
            }
        }
    }
    __syncthreads();   // `buf` is free again
}

// One tile of a fused launch: rows [row0, row1) of segment `sg` for its
// steps (plus the value pass), with the policy already in the registers of
// `mlp` and its per-feature table in LDS.
template <class E, class L, int NW>
__device__ __forceinline__ void fused_tile(const Segment& sg, int tile, L& mlp, char* smem,
                                           char* extra, char* draws, const float*& staged,
                                           int tid, int wave, int lane) {
    using HO = HeadOf<E>;
    constexpr int DT = L::DTYPE;
    constexpr int R = L::R;
    constexpr int NTHR = NW * 64;
    constexpr int G = lanes_per_row(R, NTHR, E::LANES);   // lanes serving one row in phase D
    using B = Block<E, G>;
    constexpr int C = B::C;
    static_assert(R * G <= NTHR, "G lanes per tile row");
    const int rr = tid / G, sub = tid % G;   // tile row and lane within its group
    // The action draw of a step depends only on the key, the step and the row,
    // so when whole waves are left over after the R G row lanes, R of their
    // lanes (draw lanes, starting at the next wave) compute the next step's
    // draws while the row lanes run this step's sampling and dynamics; the
    // draws pass through LDS, double-buffered by step parity. The market
    // keeps its draws on the row lanes.
    constexpr int DOFF = (R * G + 63) / 64 * 64;
    constexpr bool kDrawLanes = E::KIND != Market::KIND && E::KIND != Reaction::KIND &&
                                DOFF + R <= NTHR;
    // The reaction walk (16 lanes per row, one wave per SIMD, two Philox
    // blocks and a Box-Muller pair per step) and the market (four lanes per
    // row, one Philox block per step, two workgroups per CU bound by vector
    // instructions) draw ahead instead: every G steps, lane `sub` of a row's
    // group draws for step t + sub (the action's uniform, and the reaction's
    // energy noise), and each step takes its draws from that lane, so a step
    // pays for 1 / G of the draws. The values are the same draws.
    constexpr bool kAhead = (E::KIND == Reaction::KIND || E::KIND == Market::KIND) && G > 1;
    float ahead_u = 0.0f, ahead_z = 0.0f, noise_z = 0.0f;
    const int ahead_base = (tid & 63) & ~(G - 1);   // the group's first lane in the wave
    Pre<E>* const pbuf = reinterpret_cast<Pre<E>*>(draws);   // [2][R]
    const int dr = tid - DOFF;                               // a draw lane's tile row
    const PolicyArgs& pol = sg.pol;
    const float inv_q0 = DT == DT_FP8 ? 1.0f / pol.act_scale[0] : 1.0f;
    const float log_std = (E::NACT == 0 && pol.log_std) ? pol.log_std[0] : 0.0f;
    const int j0 = B::first(sub);
    float b3b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) b3b[c] = j0 + c < HO::NOUT ? pol.b3[j0 + c] : 0.0f;
    const float b3v = pol.b3[HO::NOUT];
    EnvCtx ctx{reinterpret_cast<const float*>(extra), nullptr, 1};
    double* const lds_cache = reinterpret_cast<double*>(extra + kRxCacheOff);   // reaction
    int* sums = reinterpret_cast<int*>(extra);   // market: [2][R][2]
    // the segment's fields the steps use, read once from LDS into scalar
    // registers (they are uniform over the workgroup)
    const EnvArgs env = uniform(sg.env);
    const GTraj tr = global_view(uniform(sg.tr));
    const int horizon = __builtin_amdgcn_readfirstlane(sg.steps);
    const RngKey key = rng_key(env);
    const uint32_t t0 = step_base(env);
    if constexpr (E::KIND == Reaction::KIND) {
        if (env.params != staged) {   // uniform over the workgroup
            stage_params(reinterpret_cast<float*>(extra), env.params, tid, NTHR);
            staged = env.params;
            __syncthreads();
        }
    }
    const Tile tl = tile_of(env, tile - __builtin_amdgcn_readfirstlane(sg.tile_begin));
    const bool mine = rr < R;
    const bool valid = mine && tl.row0 + rr < tl.row1;
    const int row = valid ? tile_row(env, tl.row0 + rr) : tl.row0 + rr;
    const bool lead = valid && sub == 0;   // writes the row's scalar records
    const int drow = tl.row0 + dr;
    const bool dvalid = kDrawLanes && dr >= 0 && dr < R && drow < tl.row1;
    // the market's lanes hold slices of the row's state (its observation is
    // the state itself); the reaction walk's lanes hold slices of its
    // coordinates (its observation) and the energy; the other kinds hold the
    // whole state on every lane
    constexpr bool kSlice = E::KIND == Market::KIND;
    constexpr bool kRx = E::KIND == Reaction::KIND && kAhead;
    static_assert(!kSlice || (E::SD % G == 0 && E::OD == E::SD), "state slices");
    constexpr int NXS = (E::OD + G - 1) / G;   // observation entries per lane
    constexpr int NS = kSlice ? E::SD / G : kRx ? NXS + 1 : E::SR;
    float s[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) s[i] = 0.0f;
    if (valid) {
        if constexpr (kSlice) load_slice<E, G>(env, row, s, sub);
        else if constexpr (kRx) load_rx_slice<G>(env, row, s, sub);
        else load_state<E>(env, row, s);
    }
    if constexpr (E::KIND == Reaction::KIND) {
        // the tile's cache into LDS (rows are consecutive for this kind)
        for (int i = tid; i < Reaction::NCACHE * R; i += NTHR) {
            const int r = i % R, j = i / R;
            if (tl.row0 + r < tl.row1)
                lds_cache[r * kRxCachePitch + j] = env.cache[(size_t)j * env.n_rows + tl.row0 + r];
        }
        ctx.cache = lds_cache + (mine ? rr : 0) * kRxCachePitch;
    }
    int slot = 0;
    if constexpr (E::KIND == Market::KIND) {
        if (valid) slot = env.slot_map[tl.row0 + rr];
        for (int i = tid; i < 4 * R; i += NTHR) sums[i] = 0;
    }
    if (mine) {
        if constexpr (kSlice || kRx) {
            L::template put_obs_slice<E::OD, G>(smem, rr, s, inv_q0, sub);
            if (valid && horizon > 0) store_obs_slice<E::OD, G>(tr.obs + (size_t)row * E::OD, s, sub);
        } else {
            float o[E::OD];
            E::observe(s, o);
            L::template put_obs<E::OD, G>(smem, rr, o, inv_q0, sub);
            if (valid && horizon > 0) store_obs<E::OD, G>(tr.obs + (size_t)row * E::OD, o, sub);
        }
    }
    const float sigma = expf(log_std);
    Pre<E> pre{0.0f, 0.0f};   // step 0's draw
    if constexpr (kDrawLanes) {
        if (dvalid) pbuf[dr] = prepare<E>(key, t0, (uint32_t)drow, log_std);
    } else if constexpr (!kAhead) {
        pre = prepare<E>(key, t0, (uint32_t)row, log_std);
    }
    __syncthreads();

    const int passes = horizon + (__builtin_amdgcn_readfirstlane(sg.last) ? 1 : 0);   // + V(s_T)
    for (int step = 0; step < passes; ++step) {
        mlp.forward(smem, wave, lane);
        __syncthreads();
        const uint32_t t = t0 + (uint32_t)step;
        const size_t idx = (size_t)step * env.n_rows + row;
        if constexpr (kDrawLanes) {   // the next step's draws, beside this step's row work
            if (dvalid && step + 1 < horizon)
                pbuf[((step + 1) & 1) * R + dr] = prepare<E>(key, t + 1, (uint32_t)drow, log_std);
        }
        if constexpr (kAhead) {   // every lane, so each source lane holds its value
            if (step % G == 0) {
                const uint32_t ts = t + (uint32_t)sub;
                ahead_u = prepare<E>(key, ts, (uint32_t)row, log_std).u;
                if constexpr (E::KIND == Reaction::KIND)
                    ahead_z = Reaction::noise_normal(key, ts + 1, (uint32_t)row);
            }
            const int src = ahead_base | (step % G);
            pre.u = __shfl(ahead_u, src);
            if constexpr (E::KIND == Reaction::KIND) noise_z = __shfl(ahead_z, src);
        }
        Act<E> act{0, 0.0f};
        // reaction: the lane's cache entries and constants, read ahead of the draw
        [[maybe_unused]] typename std::conditional<kRx, Reaction::Lane<G>, int>::type rxl{};
        if constexpr (kRx) Reaction::lane_load<G>(rxl, ctx, sub);
        if (valid) {
            float hb[C], hv;
            L::template head_block<HO::NH, C>(smem, b3b, b3v, rr, j0, hb, hv);
            if (step == horizon) {
                if (lead) tr.last_value[row] = hv;
            } else {
                float logp;
                if constexpr (kDrawLanes) pre = pbuf[(step & 1) * R + rr];
                act = decide<E, G, C>(hb, sub, pre, sigma, logp);
                if (lead) {
                    tr.value[idx] = hv;
                    tr.logp[idx] = logp;
                    store_action<E>(tr, idx, act);
                }
                if constexpr (E::KIND == Market::KIND) {
                    if (lead) {
                        int dh, s18;
                        Market::decide(act.index, dh, s18);
                        int* sl = sums + ((step & 1) * R + slot) * 2;
                        atomicAdd(sl, dh);
                        atomicAdd(sl + 1, s18);
                    }
                }
            }
        }
        if constexpr (E::KIND == Market::KIND) {
            __syncthreads();
            if (step < horizon) {
                if (valid) {
                    Pre<E> nxt{0.0f, 0.0f};
                    if constexpr (!kAhead) nxt = prepare<E>(key, t + 1, (uint32_t)row, log_std);
                    const int* sl = sums + ((step & 1) * R + slot) * 2;
                    float reward;
                    Market::settle_slice<G>(s, sub, act.index, sl[0], sl[1], reward);
                    if constexpr (!kAhead) pre = nxt;
                    if (lead) {
                        tr.reward[idx] = reward;
                        tr.done[idx] = 0;
                    }
                }
                // the other parity's sums were last read in the previous step
                for (int i = tid; i < 2 * R; i += NTHR) sums[((step + 1) & 1) * 2 * R + i] = 0;
            }
        } else if constexpr (!kSlice) {
            if (valid && step < horizon) {
                // the next step's draw, independent of this step's dynamics
                Pre<E> nxt{0.0f, 0.0f};
                if constexpr (!kDrawLanes && !kAhead)
                    nxt = prepare<E>(key, t + 1, (uint32_t)row, log_std);
                float reward;
                bool done = false;
                if constexpr (kRx)
                    Reaction::step_slice<G>(s, s[NXS], rxl, act.index, noise_z, ctx, sub,
                                            ahead_base, reward);
                else
                    E::template step<G>(s, act.index, act.value, t, (uint32_t)row, key, ctx, sub,
                                        reward, done);
                if constexpr (!kDrawLanes && !kAhead) pre = nxt;
                if (done) E::reset(s, key, t + 1, (uint32_t)row, ctx);
                if (lead) {
                    tr.reward[idx] = reward;
                    tr.done[idx] = done ? 1 : 0;
                }
            }
        }
        if (valid && step < horizon) {
            const gptr<float> dst = tr.obs + ((size_t)(step + 1) * env.n_rows + row) * E::OD;
            if constexpr (kSlice || kRx) {
                L::template put_obs_slice<E::OD, G>(smem, rr, s, inv_q0, sub);
                if (step + 1 < horizon) store_obs_slice<E::OD, G>(dst, s, sub);
            } else {
                float o[E::OD];
                E::observe(s, o);
                L::template put_obs<E::OD, G>(smem, rr, o, inv_q0, sub);
                if (step + 1 < horizon) store_obs<E::OD, G>(dst, o, sub);
            }
        }
        __syncthreads();
    }
    if (valid) {
        if constexpr (kSlice) save_slice<E, G>(env, row, s, sub);
        else if constexpr (kRx) save_rx_slice<G>(env, row, s, sub);
        else save_state<E, G>(env, row, s, sub);
    }
    if constexpr (E::KIND == Reaction::KIND) {
        __syncthreads();   // every lane's last cache update is in LDS
        for (int i = tid; i < Reaction::NCACHE * R; i += NTHR) {
            const int r = i % R, j = i / R;
            if (tl.row0 + r < tl.row1)
                env.cache[(size_t)j * env.n_rows + tl.row0 + r] = lds_cache[r * kRxCachePitch + j];
        }
    }
}

// The reset kernel's work for the rows of one tile (segments with `reset`),
// run by a fused launch before its first tile: the same draws and stores, so
// the state block ends up as the reset kernel leaves it, bit for bit.
template <class E, int NTHR>
__device__ void reset_tile(const Segment& sg, int tile, char* extra, const float*& staged,
                           int tid) {
    const EnvArgs env = uniform(sg.env);
    EnvCtx ctx{nullptr, nullptr, 0};
    if constexpr (E::KIND == Reaction::KIND) {
        if (env.params != staged) {   // uniform over the workgroup
            __syncthreads();          // earlier readers of the staged block are done
            stage_params(reinterpret_cast<float*>(extra), env.params, tid, NTHR);
            staged = env.params;
            __syncthreads();
        }
        ctx.lds_params = reinterpret_cast<const float*>(extra);
        ctx.cache_stride = (int)env.n_rows;
    }
    const Tile tl = tile_of(env, tile - __builtin_amdgcn_readfirstlane(sg.tile_begin));
    const RngKey key{env.k0, env.k1, env.epoch};
    for (int i = tl.row0 + tid; i < tl.row1; i += NTHR) {
        const int row = tile_row(env, i);
        if constexpr (E::KIND == Reaction::KIND) ctx.cache = env.cache + row;
        float s[E::SR];
        E::reset(s, key, 0u, (uint32_t)row, ctx);
        save_state<E, 1>(env, row, s, 0);
    }
}

// Persistent fused roll-out: each workgroup walks tiles of the launch's
// segments; E2 (if not E) is a second environment kind whose tiles share the
// policy shape. The weights are (re)loaded when a tile's policy differs from
// the one in the registers.
template <class E, class E2, int DT, int H, int NW, int NT, int HS, int OCC>
__global__ void __attribute__((amdgpu_flat_work_group_size(NW * 64, NW * 64),
                               amdgpu_waves_per_eu(OCC)))
k_fused(Batch batch) {
    using HO = HeadOf<E>;
    static_assert(HeadOf<E2>::NHP == HO::NHP && kin_of<E2, DT>() == kin_of<E, DT>(),
                  "kinds of one kernel share the policy shape");
    using L = Mlp<DT, H, NW, NT, kin_of<E, DT>(), HO::NHP, HS, OCC>;
    constexpr int R = L::R;
    constexpr int NTHR = NW * 64;
    constexpr int EXTRA = extra_lds_bytes<E>(R) > extra_lds_bytes<E2>(R) ? extra_lds_bytes<E>(R)
                                                                         : extra_lds_bytes<E2>(R);
    constexpr int DRAWS = 2 * R * (int)sizeof(Pre<E>);   // the draw lanes' buffer
    static_assert(sizeof(Pre<E>) == sizeof(Pre<E2>), "one draw buffer for both kinds");
    __shared__ __attribute__((aligned(16))) char smem[L::BYTES + EXTRA + DRAWS];
    char* extra = smem + L::BYTES;
    char* draws = extra + EXTRA;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    L mlp;
    int loaded = -1;                 // segment whose policy is in the registers
    const float* staged = nullptr;   // reaction: potential block now in LDS
    // zero the input tile once: its padding columns stay zero
    for (int i = tid; i < R * L::P_IN / 4; i += NTHR)
        reinterpret_cast<uint32_t*>(smem + L::OFF_IN)[i] = 0u;

    __shared__ Segment seg;          // the current tile's segment
    const int first = xcd_block();   // this workgroup's tiles: first + k * gridDim.x
    if (batch.any_reset) {
        // reset the rows of this workgroup's tiles before any weights occupy
        // registers; the tiles below read the state back (the workgroup's own
        // stores, visible after a barrier)
        for (int tile = first; tile < batch.n_tiles; tile += gridDim.x) {
            const int si = segment_index(batch, tile);
            __syncthreads();
            stage_segment(batch, si, &seg, tid, NTHR);
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(seg.reset)) {
                if constexpr (!std::is_same<E, E2>::value) {
                    if (seg.env.kind == E2::KIND) {
                        reset_tile<E2, NTHR>(seg, tile, extra, staged, tid);
                        continue;
                    }
                }
                reset_tile<E, NTHR>(seg, tile, extra, staged, tid);
            }
        }
    }
    for (int tile = first; tile < batch.n_tiles; tile += gridDim.x) {
        const int si = segment_index(batch, tile);   // uniform over the workgroup
        __syncthreads();   // the previous tile's last reads of `seg` and the table are done
        stage_segment(batch, si, &seg, tid, NTHR);
        __syncthreads();
        const Segment& sg = seg;
        if (si != loaded) {
            mlp.load(sg.pol, smem, wave, lane, tid);
            loaded = si;
            __syncthreads();
        }
        if constexpr (!std::is_same<E, E2>::value) {
            if (sg.env.kind == E2::KIND) {
                fused_tile<E2, L, NW>(sg, tile, mlp, smem, extra, draws, staged, tid, wave, lane);
                continue;
            }
        }
        fused_tile<E, L, NW>(sg, tile, mlp, smem, extra, draws, staged, tid, wave, lane);
    }
    if (batch.any_gae) {
        // returns and GAE of every tile this workgroup rolled out, after all of
        // them (the weights are no longer needed, so this pass takes no
        // registers from the roll-out), with the whole LDS as its buffer
        static_assert(L::BYTES >= 32 * R, "one segment per row fits");
        for (int tile = first; tile < batch.n_tiles; tile += gridDim.x) {
            const int si = segment_index(batch, tile);
            __syncthreads();   // the previous pass over `seg` and the buffer is done
            stage_segment(batch, si, &seg, tid, NTHR);
            __syncthreads();   // also: this workgroup's records are visible to every wave
            const GaeArgs gae = uniform(seg.gae);
            if (gae.ret == nullptr) continue;
            const EnvArgs env = uniform(seg.env);
            const GTraj tr = global_view(uniform(seg.tr));
            const Tile tl = tile_of(env, tile - __builtin_amdgcn_readfirstlane(seg.tile_begin));
            // blocks of 36 steps hold a 200-step horizon's segments over
            // six row groups; kernels that keep fewer registers free for
            // this pass (their occupancy is set by the roll-out) take 16
            constexpr int GB = DT == DT_BF16 ? 36 : 16;
            tile_gae<NTHR, GB>(env, tr, gae, tl, __builtin_amdgcn_readfirstlane(seg.steps),
                               reinterpret_cast<double*>(smem), L::BYTES, tid);
        }
    }
}

// ------------------------------------------- one wave per row (FP32) --
// For a small FP32 policy (CartPole's 4-64-64-3) a 16-row MFMA tile that
// holds a few replicas wastes most of its products, and each step pays three
// workgroup barriers. This form gives a one-wave workgroup one row at a time:
// lane j owns hidden feature j of both layers (its rows of W1 and W2 and its
// column of the head in registers), the layers are FP32 FMAs, the hidden
// activations pass between the wave's lanes through 256 bytes of LDS, and
// the head is a butterfly sum over the lanes. Every lane then holds the same
// head, so the per-row phase runs on all lanes with the same values and a
// step needs no barrier.
__device__ __forceinline__ float wave_sum(float v) {
    v = group_sum<16>(v);   // every lane of 16-lane row k: its sum r_k
    // row_bcast:15 adds lane 15's r0 into row 1 and lane 47's r2 into row 3,
    // row_bcast:31 adds lane 31's r0 + r1 into row 3: lane 63 holds
    // (r3 + r2) + (r1 + r0), read into a scalar register for every lane
    v += dpp_f_rows<0x142, 0xA>(v);
    v += dpp_f_rows<0x143, 0xC>(v);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

template <class E, int H>
struct RowMlp {
    static_assert(H == 64, "one lane per hidden feature");
    using HO = HeadOf<E>;
    static constexpr int OD = E::OD, NH = HO::NH;
    float w1[OD], w2[H], w3[NH], b3[NH];
    float b1, b2;

    __device__ void load(const PolicyArgs& p, int lane) {
        const float* W1 = static_cast<const float*>(p.w1);
        const float* W2 = static_cast<const float*>(p.w2);
        const float* W3 = static_cast<const float*>(p.w3);
#pragma unroll
        for (int k = 0; k < OD; ++k) w1[k] = W1[lane * p.d_in + k];
#pragma unroll
        for (int k = 0; k < H; ++k) w2[k] = W2[lane * H + k];
#pragma unroll
        for (int o = 0; o < NH; ++o) {
            w3[o] = W3[o * H + lane];
            b3[o] = p.b3[o];
        }
        b1 = p.b1[lane];
        b2 = p.b2[lane];
    }

    // Head outputs for observation `o` (the same on every lane) and this
    // lane's hidden activations; `lds` holds H floats private to the wave.
    __device__ void forward(const float (&o)[OD], float* lds, int lane, float (&head)[NH],
                            float& h1, float& h2) const {
        float z1 = b1;
#pragma unroll
        for (int k = 0; k < OD; ++k) z1 = __builtin_fmaf(w1[k], o[k], z1);
        h1 = tanh_scaled(z1, kTwoLog2e);
        lds[lane] = h1;
        wave_lds_sync();
        float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // k mod 8
#pragma unroll
        for (int k4 = 0; k4 < H / 4; ++k4) {
            const float4 v = reinterpret_cast<const float4*>(lds)[k4];
            const int c = 4 * (k4 & 1);
            acc[c + 0] = __builtin_fmaf(w2[4 * k4 + 0], v.x, acc[c + 0]);
            acc[c + 1] = __builtin_fmaf(w2[4 * k4 + 1], v.y, acc[c + 1]);
            acc[c + 2] = __builtin_fmaf(w2[4 * k4 + 2], v.z, acc[c + 2]);
            acc[c + 3] = __builtin_fmaf(w2[4 * k4 + 3], v.w, acc[c + 3]);
        }
        const float z2 = b2 + (((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                               ((acc[4] + acc[5]) + (acc[6] + acc[7])));
        h2 = tanh_scaled(z2, kTwoLog2e);
#pragma unroll
        for (int j = 0; j < NH; ++j) head[j] = b3[j] + wave_sum(w3[j] * h2);
    }
};

// The row-per-wave form over the tiles (rows) of a launch's segments, with
// the same reset pre-pass and returns post-pass as k_fused.
template <class E, int H>
__global__ void __launch_bounds__(64) k_fused_rw(Batch batch) {
    using HO = HeadOf<E>;
    using B = Block<E, 1>;
    constexpr int C = B::C;
    static_assert(E::LANES == 1, "one-lane environments");
    __shared__ __attribute__((aligned(16))) char smem[64 * 32];   // h1, then the returns' buffer
    __shared__ Segment seg;
    float* h1s = reinterpret_cast<float*>(smem);
    const int lane = threadIdx.x;
    const float* staged = nullptr;
    const int first = xcd_block();   // this workgroup's rows: first + k * gridDim.x
    if (batch.any_reset) {
        for (int tile = first; tile < batch.n_tiles; tile += gridDim.x) {
            const int si = segment_index(batch, tile);
            __syncthreads();
            stage_segment(batch, si, &seg, lane, 64);
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(seg.reset)) reset_tile<E, 64>(seg, tile, smem, staged, lane);
        }
    }
    RowMlp<E, H> mlp;
    int loaded = -1;
    for (int tile = first; tile < batch.n_tiles; tile += gridDim.x) {
        const int si = segment_index(batch, tile);
        __syncthreads();
        stage_segment(batch, si, &seg, lane, 64);
        __syncthreads();
        const EnvArgs env = uniform(seg.env);
        const GTraj tr = global_view(uniform(seg.tr));
        const PolicyArgs& pol = seg.pol;
        if (si != loaded) {
            mlp.load(pol, lane);
            loaded = si;
        }
        const int horizon = __builtin_amdgcn_readfirstlane(seg.steps);
        const int passes = horizon + (__builtin_amdgcn_readfirstlane(seg.last) ? 1 : 0);
        const RngKey key = rng_key(env);
        const uint32_t t0 = step_base(env);
        const Tile tl = tile_of(env, tile - __builtin_amdgcn_readfirstlane(seg.tile_begin));
        if (tl.row0 >= tl.row1) continue;
        const int row = tile_row(env, tl.row0);
        const float log_std = (E::NACT == 0 && pol.log_std) ? pol.log_std[0] : 0.0f;
        const float sigma = expf(log_std);
        EnvCtx ctx{nullptr, nullptr, 1};
        float s[E::SR];
        load_state<E>(env, row, s);
        float o[E::OD];
        E::observe(s, o);
        if (horizon > 0) {
            float ok = 0.0f;
#pragma unroll
            for (int k = 0; k < E::OD; ++k) ok = lane == k ? o[k] : ok;
            if (lane < E::OD) tr.obs[(size_t)row * E::OD + lane] = ok;
        }
        // the draws of the next 64 steps, one per lane, taken with readlane
        Pre<E> ahead{0.0f, 0.0f};
        for (int step = 0; step < passes; ++step) {
            const uint32_t t = t0 + (uint32_t)step;
            if (step % 64 == 0) ahead = prepare<E>(key, t + (uint32_t)lane, (uint32_t)row, log_std);
            float head[HO::NH], h1, h2;
            mlp.forward(o, h1s, lane, head, h1, h2);
            const float hv = head[HO::NOUT];
            if (step == horizon) {
                if (lane == 0) tr.last_value[row] = hv;
                break;
            }
            Pre<E> pre;
            pre.u = __builtin_bit_cast(float, __builtin_amdgcn_readlane(
                                                  __builtin_bit_cast(int, ahead.u), step % 64));
            pre.logp = __builtin_bit_cast(float, __builtin_amdgcn_readlane(
                                                     __builtin_bit_cast(int, ahead.logp), step % 64));
            float hb[C];
#pragma unroll
            for (int c = 0; c < C; ++c) hb[c] = c < HO::NOUT ? head[c] : 0.0f;
            float logp;
            const Act<E> act = decide<E, 1, C>(hb, 0, pre, sigma, logp);
            const size_t idx = (size_t)step * env.n_rows + row;
            float reward;
            bool done;
            E::template step<1>(s, act.index, act.value, t, (uint32_t)row, key, ctx, 0, reward, done);
            if (done) E::reset(s, key, t + 1, (uint32_t)row, ctx);
            if (lane == 0) {
                tr.value[idx] = hv;
                tr.logp[idx] = logp;
                store_action<E>(tr, idx, act);
                tr.reward[idx] = reward;
                tr.done[idx] = done ? 1 : 0;
            }
            E::observe(s, o);
            if (step + 1 < horizon) {
                float ok = 0.0f;
#pragma unroll
                for (int k = 0; k < E::OD; ++k) ok = lane == k ? o[k] : ok;
                if (lane < E::OD) tr.obs[((size_t)(step + 1) * env.n_rows + row) * E::OD + lane] = ok;
            }
        }
        if (lane == 0) save_state<E, 1>(env, row, s, 0);
    }
    if (batch.any_gae) {
        for (int tile = first; tile < batch.n_tiles; tile += gridDim.x) {
            const int si = segment_index(batch, tile);
            __syncthreads();
            stage_segment(batch, si, &seg, lane, 64);
            __syncthreads();
            const GaeArgs gae = uniform(seg.gae);
            if (gae.ret == nullptr) continue;
            const EnvArgs env = uniform(seg.env);
            const GTraj tr = global_view(uniform(seg.tr));
            const Tile tl = tile_of(env, tile - __builtin_amdgcn_readfirstlane(seg.tile_begin));
            tile_gae<64, 16>(env, tr, gae, tl, __builtin_amdgcn_readfirstlane(seg.steps),
                             reinterpret_cast<double*>(smem), (int)sizeof(smem), lane);
        }
    }
}

// The row-per-wave policy alone, one row per workgroup (the plain form's
// policy step and the checker's trace): the same RowMlp code as k_fused_rw.
template <class E, int H, bool TRACE>
__device__ __forceinline__ void policy_row_rw(const EnvArgs& env, const PolicyArgs& pol, float* a1,
                                              float* a2) {
    using HO = HeadOf<E>;
    __shared__ __attribute__((aligned(16))) float h1s[H];
    const int lane = threadIdx.x;
    const int64_t row = blockIdx.x;
    if (row >= env.n_rows) return;
    RowMlp<E, H> mlp;
    mlp.load(pol, lane);
    float o[E::OD];
#pragma unroll
    for (int k = 0; k < E::OD; ++k) o[k] = env.obs_scratch[(size_t)row * E::OD + k];
    float head[HO::NH], h1, h2;
    mlp.forward(o, h1s, lane, head, h1, h2);
    if constexpr (TRACE) {
        a1[(size_t)row * H + lane] = h1;
        a2[(size_t)row * H + lane] = h2;
    }
    float hj = 0.0f;
#pragma unroll
    for (int j = 0; j < HO::NH; ++j) hj = lane == j ? head[j] : hj;
    if (lane < HO::NH) env.head_scratch[(size_t)row * HO::NH + lane] = hj;
}

// -------------------------------------------------------------- reset --
template <class E>
__global__ void k_reset(EnvArgs env) {
    __shared__ float params[E::KIND == Reaction::KIND ? Reaction::PARAM_FLOATS : 1];
    EnvCtx ctx{nullptr, nullptr, 0};
    if constexpr (E::KIND == Reaction::KIND) {
        stage_params(params, env.params, threadIdx.x, blockDim.x);
        ctx.lds_params = params;
    }
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= env.n_rows) return;
    if constexpr (E::KIND == Reaction::KIND) {
        ctx.cache = env.cache + row;
        ctx.cache_stride = (int)env.n_rows;
    }
    const RngKey key{env.k0, env.k1, env.epoch};
    float s[E::SR];
    E::reset(s, key, 0u, (uint32_t)row, ctx);
    save_state<E, 1>(env, row, s, 0);
}

}  // namespace wsx
