// update.hip -- actor-critic gradient and Adam on the device (arXiv
// 2408.00930, Sec. 3: actor-critic training for discrete and continuous
// actions on the roll-out data kept in device memory; App. A: the trainer
// consumes the roll-out where it was written).
//
// Loss (a reading: the paper names the method, not the loss), averaged over
// the n samples (horizon x rows of one trajectory):
//   L = (1/n) sum_i [ -A_i log pi(a_i|o_i) + (c_v/2) (V(o_i) - G_i)^2 - c_e H(pi(.|o_i)) ]
// The policy is evaluated as the roll-out evaluates it (BF16 or FP32 inputs
// of every product, FP32 accumulation) and the gradient passes the rounding
// straight through, the derivative of tanh taken at the unrounded FP32
// activation. The operands of the backward products are rounded to the
// policy's format: the head gradient before it meets W3 and h2, dz2 and dz1
// before they meet the weights and the layer inputs; bias gradients sum the
// unrounded values.
//
// Three kernels:
//  k_ac_fwd   per 32-sample tile: forward (layer 1, layer 2, head), head
//             gradient, dz2 = (dhead W3) (1 - t2^2); accumulates dW3, db3,
//             db2 and the log-std gradient; writes the dz2 rows to the
//             workspace (the only per-sample staging, written once, read
//             once).
//  k_ac_bwd   per tile: layer 1 again, dz1 = (dz2 W2) (1 - t1^2) with W2's
//             columns in LDS, dW1 and db1, and dW2 = sum_i dz2_i h1_i^T
//             with h1 from the accumulators and dz2 read down the columns of
//             its rows in LDS, split over the samples (split-K).
//  k_ac_sum   per-workgroup partial sums -> the gradients, one launch.
// The products run with samples as the MFMA rows (the weight fragments the
// roll-out loads as A operands serve unchanged as B operands), so the
// accumulators hold [sample][feature] tiles: lane l has feature l mod 16 and
// samples 4 (l / 16) + i of each 16-sample row tile. Those tiles feed the
// weight-gradient products (K = samples) directly, taking the K elements in
// accumulator order; the other operand is read from LDS in the same order.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace wsx {

namespace {

constexpr int kAcRows = 32;   // samples per tile (two row tiles of 16)
// samples per pass over the workspace: larger sets run in chunks, so the
// workspace stays bounded (1 GiB for BF16 hidden 256)
constexpr int64_t kAcChunk = int64_t(1) << 21;

// KC elements of a B fragment down column `col` of a row-major [k][ld]
// matrix: W[(k0 + e) * ld + col], zero for rows >= k_valid.
__device__ __forceinline__ void load_col(float& f, const void* W, int ld, int col, int k0,
                                         int k_valid) {
    const float* w = static_cast<const float*>(W);
    f = k0 < k_valid ? w[(size_t)k0 * ld + col] : 0.0f;
}
__device__ __forceinline__ void load_col(bf16x8& f, const void* W, int ld, int col, int k0,
                                         int k_valid) {
    const uint16_t* w = static_cast<const uint16_t*>(W);
    uint16_t v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
        v[e] = k0 + e < k_valid ? w[(size_t)(k0 + e) * ld + col] : (uint16_t)0;
    __builtin_memcpy(&f, v, 16);
}

template <int DT>
__device__ __forceinline__ float round_to(float x) {
    if constexpr (DT == DT_BF16) return (float)(__bf16)x;
    return x;
}

// One element of the policy format at byte address p (rounded to nearest
// even for BF16).
template <int DT>
__device__ __forceinline__ void put(char* p, float v) {
    if constexpr (DT == DT_BF16)
        *reinterpret_cast<__bf16*>(p) = (__bf16)v;
    else
        *reinterpret_cast<float*>(p) = v;
}

// BF16 fragment whose K elements are samples in accumulator order: elements
// 0-3 are row tile 0's i = 0..3, elements 4-7 row tile 1's.
__device__ __forceinline__ bf16x8 pack_acc_k(const f32x4& a0, const f32x4& a1) {
    const uint4 u = make_uint4(pack_bf16x2(a0[0], a0[1]), pack_bf16x2(a0[2], a0[3]),
                               pack_bf16x2(a1[0], a1[1]), pack_bf16x2(a1[2], a1[3]));
    return __builtin_bit_cast(bf16x8, u);
}

// The matching BF16 fragment from a transposed LDS tile T[c][sample]: row c,
// samples 4 q .. 4 q + 3 and 16 + 4 q .. 16 + 4 q + 3.
__device__ __forceinline__ bf16x8 lds_k_perm(const char* T, int pitch, int c, int q) {
    const uint2 lo = *reinterpret_cast<const uint2*>(T + c * pitch + (4 * q) * 2);
    const uint2 hi = *reinterpret_cast<const uint2*>(T + c * pitch + (16 + 4 * q) * 2);
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

// The same fragment from a row-major LDS tile T[sample][column]: column c,
// the same samples, eight 16-bit reads down the column.
__device__ __forceinline__ bf16x8 lds_col_perm(const char* T, int pitch, int c, int q) {
    uint16_t v[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = *reinterpret_cast<const uint16_t*>(T + (4 * q + i) * pitch + c * 2);
        v[4 + i] = *reinterpret_cast<const uint16_t*>(T + (16 + 4 * q + i) * pitch + c * 2);
    }
    bf16x8 f;
    __builtin_memcpy(&f, v, 16);
    return f;
}

__device__ __forceinline__ float act_tanh(float z) { return tanh_scaled(z, kTwoLog2e); }

// Workgroup barrier for LDS traffic only: this wave's LDS operations complete,
// then s_barrier. Unlike __syncthreads() it does not wait for the wave's
// global loads and stores, so loads issued for the next tile stay in flight
// across it (no wave reads another wave's global writes inside these kernels).
__device__ __forceinline__ void lds_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

// A workgroup's partial sum: written by the first chunk of samples, added to
// by later chunks (each workgroup owns its slot; chunks run in stream order).
__device__ __forceinline__ void part_out(float* p, float v, bool acc) { *p = acc ? *p + v : v; }

template <int DT, int H, int KIN, int NHP>
struct AcShape {
    using M = Mma<DT>;
    using Frag = typename M::frag;
    static constexpr int K = M::K, KC = M::KC, EB = M::EB;
    static constexpr int NW = H >= 256 ? 8 : H / 16;   // waves; each owns FPW features
    static constexpr int NTHR = NW * 64;
    static constexpr int FPW = H / NW, MT = FPW / 16;
    static constexpr int K1S = KIN / K, K2S = H / K;
    static constexpr int NHT = NHP / 16;
    static constexpr int NHK = (NHP + K - 1) / K * K;   // head width padded to K
    static constexpr int KO = NHK / K;
    static constexpr int KT = (KIN + 15) / 16;          // 16-column tiles of dW1
    static constexpr int R = kAcRows;
    static constexpr int P_IN = KIN * EB + 16, P_H = H * EB + 16, P_DH = NHK * EB + 16;
    static constexpr int P_T = R * EB + 16;   // transposed tiles: [feature][sample]
    static constexpr int KINP = KIN;
    static constexpr int FWD_FLOATS = NHP * H + H + NHP + 1;   // dW3, db2, db3, dlog_std
    static constexpr int BWD_FLOATS = H * KIN + H;             // dW1, db1
    static_assert(FPW % 16 == 0 && H % K == 0 && KIN % K == 0, "tile shape");
    static_assert(NHT * 2 <= NW, "one wave per head tile and row tile");
};

// Observation elements of a tile, loaded into registers one tile ahead (the
// load latency hides behind the current tile), then stored into LDS rows (and
// their transpose if x0T is set); zero beyond d_in and beyond n.
template <class S>
struct ObsPrefetch {
    static constexpr int KIN = S::KINP;
    static constexpr int PER = (S::R * KIN + S::NTHR - 1) / S::NTHR;
    float v[PER];
    __device__ __forceinline__ void load(const AcArgs& a, int64_t tile, int tid) {
        const int d_in = a.pol.d_in;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * S::NTHR;
            const int r = e / KIN, i = e % KIN;
            const int64_t n = tile * S::R + r;
            v[u] = (e < S::R * KIN && n < a.n && i < d_in) ? a.obs[n * d_in + i] : 0.0f;
        }
    }
    template <int DT>
    __device__ __forceinline__ void store(char* x0, char* x0T, int tid) const {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * S::NTHR;
            if (e >= S::R * KIN) break;
            const int r = e / KIN, i = e % KIN;
            put<DT>(x0 + r * S::P_IN + i * S::EB, v[u]);
            if (x0T) put<DT>(x0T + i * S::P_T + r * S::EB, v[u]);
        }
    }
};

template <int DT, int H, int KIN, int NHP>
__global__ void __launch_bounds__((AcShape<DT, H, KIN, NHP>::NTHR))
k_ac_fwd(AcArgs a) {
    using S = AcShape<DT, H, KIN, NHP>;
    using M = typename S::M;
    using Frag = typename S::Frag;
    constexpr int R = S::R, MT = S::MT, K = S::K, KC = S::KC, EB = S::EB;
    __shared__ __attribute__((aligned(16))) char x0[R * S::P_IN];
    __shared__ __attribute__((aligned(16))) char h1[R * S::P_H];
    __shared__ __attribute__((aligned(16))) char h2[R * S::P_H];
    __shared__ __attribute__((aligned(16))) char dz[R * S::P_H];
    __shared__ __attribute__((aligned(16))) char dh[R * S::P_DH];
    __shared__ __attribute__((aligned(16))) char dhT[NHP * S::P_T];
    __shared__ float hd[R][NHP + 1];
    __shared__ float db3p[R][NHP + 1];   // per sample lane: sums over its samples
    __shared__ float dlsp[R];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, q = lane >> 4;
    const int kq = q * KC;
    const PolicyArgs& p = a.pol;
    // weights: layer 1 and 2 rows of this wave's features (B operands), the
    // head's columns of these features (B of the dz2 product), and the head
    // rows of this wave's head job
    Frag w1[MT][S::K1S], w2[MT][S::K2S], w3t[MT][S::KO], w3[S::K2S];
    float b1v[MT], b2v[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int f = wave * S::FPW + mt * 16 + lr;
#pragma unroll
        for (int ks = 0; ks < S::K1S; ++ks) load_a(w1[mt][ks], p.w1, p.d_in, f, H, ks * K + kq, p.d_in);
#pragma unroll
        for (int ks = 0; ks < S::K2S; ++ks) load_a(w2[mt][ks], p.w2, H, f, H, ks * K + kq, H);
#pragma unroll
        for (int ks = 0; ks < S::KO; ++ks) load_col(w3t[mt][ks], p.w3, H, f, ks * K + kq, p.n_head);
        b1v[mt] = p.b1[f];
        b2v[mt] = p.b2[f];
    }
    const bool head_job = wave < S::NHT * 2;
    const int jht = wave >> 1, jnt = wave & 1;
#pragma unroll
    for (int ks = 0; ks < S::K2S; ++ks)
        load_a(w3[ks], p.w3, H, head_job ? jht * 16 + lr : p.n_head, p.n_head, ks * K + kq, H);
    const float b3v = (head_job && jht * 16 + lr < p.n_head) ? p.b3[jht * 16 + lr] : 0.0f;
    const float log_std = a.n_act == 0 ? p.log_std[0] : 0.0f;
    const float sigma = expf(log_std);

    f32x4 dw3[S::NHT][MT];
    float db2a[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        db2a[mt] = 0.0f;
#pragma unroll
        for (int ht = 0; ht < S::NHT; ++ht) dw3[ht][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    for (int e = tid; e < R * (NHP + 1); e += S::NTHR) db3p[e / (NHP + 1)][e % (NHP + 1)] = 0.0f;
    if (tid < R) dlsp[tid] = 0.0f;
    // head-gradient padding (columns >= n_head) stays zero
    for (int e = tid; e < R * S::NHK; e += S::NTHR) put<DT>(dh + (e / S::NHK) * S::P_DH + (e % S::NHK) * EB, 0.0f);
    for (int e = tid; e < NHP * R; e += S::NTHR) put<DT>(dhT + (e / R) * S::P_T + (e % R) * EB, 0.0f);

    const int64_t n_tiles = (a.n + R - 1) / R;
    ObsPrefetch<S> obs;
    obs.load(a, blockIdx.x, tid);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile * R;
        lds_barrier();   // the previous tile's LDS reads are done
        obs.template store<DT>(x0, nullptr, tid);
        lds_barrier();
        // this tile's per-sample inputs (used after the head) and the next
        // tile's observations, in flight while the layers run
        float s_adv = 0.0f, s_ret = 0.0f, s_act = 0.0f;
        if (tid < R && base + tid < a.n) {
            const int64_t n = base + tid;
            s_adv = a.adv[n];
            s_ret = a.ret[n];
            s_act = a.n_act == 0 ? static_cast<const float*>(a.action)[n]
                                 : (float)static_cast<const uint8_t*>(a.action)[n];
        }
        obs.load(a, tile + gridDim.x, tid);
        // layer 1
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int f = wave * S::FPW + mt * 16 + lr;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                f32x4 acc = {b1v[mt], b1v[mt], b1v[mt], b1v[mt]};
#pragma unroll
                for (int ks = 0; ks < S::K1S; ++ks)
                    acc = M::mma(M::lds(x0 + (nt * 16 + lr) * S::P_IN + (ks * K + kq) * EB), w1[mt][ks], acc);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    put<DT>(h1 + (nt * 16 + 4 * q + i) * S::P_H + f * EB, act_tanh(acc[i]));
            }
        }
        lds_barrier();
        // layer 2, keeping the unrounded activations
        f32x4 t2[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int f = wave * S::FPW + mt * 16 + lr;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                f32x4 acc = {b2v[mt], b2v[mt], b2v[mt], b2v[mt]};
#pragma unroll
                for (int ks = 0; ks < S::K2S; ++ks)
                    acc = M::mma(M::lds(h1 + (nt * 16 + lr) * S::P_H + (ks * K + kq) * EB), w2[mt][ks], acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    t2[mt][nt][i] = act_tanh(acc[i]);
                    put<DT>(h2 + (nt * 16 + 4 * q + i) * S::P_H + f * EB, t2[mt][nt][i]);
                }
            }
        }
        lds_barrier();
        // head: wave (ht, nt) of the 2 NHT jobs
        if (head_job) {
            f32x4 acc = {b3v, b3v, b3v, b3v};
#pragma unroll
            for (int ks = 0; ks < S::K2S; ++ks)
                acc = M::mma(M::lds(h2 + (jnt * 16 + lr) * S::P_H + (ks * K + kq) * EB), w3[ks], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) hd[jnt * 16 + 4 * q + i][jht * 16 + lr] = acc[i];
        }
        lds_barrier();
        // gradient of the loss at the head, one thread per sample
        if (tid < R) {
            const int r = tid;
            const int64_t n = base + r;
            const bool ok = n < a.n;
            const float A = s_adv;
            const int NH = p.n_head;
            auto set = [&](int o, float g) {
                db3p[r][o] += g;
                const float gq = round_to<DT>(g);
                put<DT>(dh + r * S::P_DH + o * EB, gq);
                put<DT>(dhT + o * S::P_T + r * EB, gq);
            };
            if (a.n_act == 0) {
                const float mu = hd[r][0];
                const float act = ok ? s_act : mu;
                const float d = (act - mu) / sigma;
                set(0, ok ? -A * d / sigma * a.inv_n : 0.0f);
                if (ok) dlsp[r] += (-A * (d * d - 1.0f) - a.entropy_coef) * a.inv_n;
            } else {
                const int KA = a.n_act;
                float mx = hd[r][0];
                for (int k = 1; k < KA; ++k) mx = fmaxf(mx, hd[r][k]);
                float z = 0.0f;
                for (int k = 0; k < KA; ++k) z += expf(hd[r][k] - mx);
                const float lz = logf(z);
                float ent = 0.0f;
                for (int k = 0; k < KA; ++k) {
                    const float lp = hd[r][k] - mx - lz;
                    ent -= expf(lp) * lp;
                }
                const int act = ok ? (int)s_act : -1;
                for (int k = 0; k < KA; ++k) {
                    const float lp = hd[r][k] - mx - lz, pk = expf(lp);
                    const float g = (A * (pk - (k == act ? 1.0f : 0.0f)) + a.entropy_coef * pk * (lp + ent)) *
                                    a.inv_n;
                    set(k, ok ? g : 0.0f);
                }
            }
            set(NH - 1, ok ? a.value_coef * (hd[r][NH - 1] - s_ret) * a.inv_n : 0.0f);
        }
        lds_barrier();
        // dz2 = (dhead W3) (1 - t2^2) for this wave's features; dW3 += dhead^T h2
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int f = wave * S::FPW + mt * 16 + lr;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < S::KO; ++ks)
                    acc = M::mma(M::lds(dh + (nt * 16 + lr) * S::P_DH + (ks * K + kq) * EB), w3t[mt][ks], acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float t = t2[mt][nt][i];
                    const float g = acc[i] * (1.0f - t * t);
                    db2a[mt] += g;
                    put<DT>(dz + (nt * 16 + 4 * q + i) * S::P_H + f * EB, g);
                }
            }
#pragma unroll
            for (int ht = 0; ht < S::NHT; ++ht) {
                if constexpr (DT == DT_BF16) {
                    const Frag A_ = lds_k_perm(dhT, S::P_T, ht * 16 + lr, q);
                    const Frag B_ = pack_acc_k(t2[mt][0], t2[mt][1]);
                    dw3[ht][mt] = M::mma(A_, B_, dw3[ht][mt]);
                } else {
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float A_ = *reinterpret_cast<const float*>(
                                dhT + (ht * 16 + lr) * S::P_T + (16 * nt + 4 * q + i) * EB);
                            dw3[ht][mt] = M::mma(A_, t2[mt][nt][i], dw3[ht][mt]);
                        }
                }
            }
        }
        lds_barrier();
        // dz2 rows of the tile to the workspace (consecutive samples)
        const int rows = (int)min((int64_t)R, a.n - base);
        constexpr int CH = H * EB / 16;
        for (int e = tid; e < rows * CH; e += S::NTHR) {
            const int r = e / CH, c = e % CH;
            const size_t off = (size_t)(base + r) * (H * EB) + (size_t)c * 16;
            *reinterpret_cast<uint4*>(a.dz2_rows + off) =
                *reinterpret_cast<const uint4*>(dz + r * S::P_H + c * 16);
        }
    }
    // this workgroup's partial sums
    float* out = a.part_fwd + (size_t)blockIdx.x * S::FWD_FLOATS;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int f = wave * S::FPW + mt * 16 + lr;
#pragma unroll
        for (int ht = 0; ht < S::NHT; ++ht)
#pragma unroll
            for (int i = 0; i < 4; ++i) part_out(&out[(ht * 16 + 4 * q + i) * H + f], dw3[ht][mt][i], a.accumulate);
        float v = db2a[mt];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (q == 0) part_out(&out[NHP * H + f], v, a.accumulate);
    }
    lds_barrier();
    if (tid < NHP) {
        float v = 0.0f;
        for (int r = 0; r < R; ++r) v += db3p[r][tid];
        part_out(&out[NHP * H + H + tid], v, a.accumulate);
    }
    if (tid == 0) {
        float v = 0.0f;
        for (int r = 0; r < R; ++r) v += dlsp[r];
        part_out(&out[NHP * H + H + NHP], v, a.accumulate);
    }
}

// The backward pass of a tile after the forward kernel, from the tile's dz2
// rows (read once) and its observations: layer 1 again (h1 of this wave's
// features: unrounded for tanh', rounded as the forward rounded it for dW2),
// dh1 = dz2 W2 with W2's columns at this wave's features as B fragments,
// dz1 = dh1 (1 - t1^2), dW1 += dz1^T x0 and db1, and dW2 += dz2^T h1 with h1
// from the accumulators as B fragments (K = the tile's samples in
// accumulator order) and each dz2 column's A fragment read down the tile's
// rows in the same sample order. The dW2 partial sums (all of dW2's rows at
// this wave's columns) stay in registers for the whole launch, so W2's
// columns live in LDS instead ([wave][mt][ks][lane] fragments, written once
// per workgroup). The next tile's observations and dz2 rows are loaded into
// registers while the current one runs; two barriers per tile.
template <int DT, int H, int KIN, int NHP>
__global__ void __launch_bounds__((AcShape<DT, H, KIN, NHP>::NTHR))
k_ac_bwd(AcArgs a) {
    using S = AcShape<DT, H, KIN, NHP>;
    using M = typename S::M;
    using Frag = typename S::Frag;
    constexpr int R = S::R, MT = S::MT, K = S::K, KC = S::KC, EB = S::EB, NJT = H / 16;
    constexpr int NW = S::NTHR / 64;
    __shared__ __attribute__((aligned(16))) Frag w2tl[NW * MT * S::K2S * 64];
    __shared__ __attribute__((aligned(16))) char x0[R * S::P_IN];
    __shared__ __attribute__((aligned(16))) char x0T[S::KT * 16 * S::P_T];
    __shared__ __attribute__((aligned(16))) char dzs[R * S::P_H];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, q = lane >> 4;
    const int kq = q * KC;
    const PolicyArgs& p = a.pol;
    auto w2t = [&](int mt, int ks) -> Frag& {
        return w2tl[((wave * MT + mt) * S::K2S + ks) * 64 + lane];
    };
    Frag w1[MT][S::K1S];
    float b1v[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int f = wave * S::FPW + mt * 16 + lr;
#pragma unroll
        for (int ks = 0; ks < S::K1S; ++ks) load_a(w1[mt][ks], p.w1, p.d_in, f, H, ks * K + kq, p.d_in);
#pragma unroll
        for (int ks = 0; ks < S::K2S; ++ks) load_col(w2t(mt, ks), p.w2, H, f, ks * K + kq, H);
        b1v[mt] = p.b1[f];
    }
    f32x4 dw1[MT][S::KT], acc[NJT][MT];
    float db1a[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        db1a[mt] = 0.0f;
#pragma unroll
        for (int it = 0; it < S::KT; ++it) dw1[mt][it] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int jt = 0; jt < NJT; ++jt) acc[jt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // transposed-input rows >= KIN stay zero
    for (int e = tid; e < (S::KT * 16 - KIN) * R; e += S::NTHR)
        put<DT>(x0T + (KIN + e / R) * S::P_T + (e % R) * EB, 0.0f);

    const int64_t n_tiles = (a.n + R - 1) / R;
    constexpr int CH = H * EB / 16;
    constexpr int DPER = (R * CH + S::NTHR - 1) / S::NTHR;
    uint4 dzv[DPER];
    auto load_dz = [&](int64_t tile) {
#pragma unroll
        for (int u = 0; u < DPER; ++u) {
            const int e = tid + u * S::NTHR;
            const int r = e / CH, c = e % CH;
            const int64_t n = tile * R + r;
            dzv[u] = make_uint4(0u, 0u, 0u, 0u);
            if (e < R * CH && n < a.n)
                dzv[u] = *reinterpret_cast<const uint4*>(a.dz2_rows + (size_t)n * (H * EB) +
                                                         (size_t)c * 16);
        }
    };
    ObsPrefetch<S> obs;
    obs.load(a, blockIdx.x, tid);
    load_dz(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        lds_barrier();   // the previous tile's reads of the buffers are done
        obs.template store<DT>(x0, x0T, tid);
#pragma unroll
        for (int u = 0; u < DPER; ++u) {
            const int e = tid + u * S::NTHR;
            if (e < R * CH) *reinterpret_cast<uint4*>(dzs + (e / CH) * S::P_H + (e % CH) * 16) = dzv[u];
        }
        obs.load(a, tile + gridDim.x, tid);
        load_dz(tile + gridDim.x);
        lds_barrier();
        f32x4 t[MT][2];   // h1 of this wave's features, unrounded
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f32x4 g[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                f32x4 z = {b1v[mt], b1v[mt], b1v[mt], b1v[mt]};
#pragma unroll
                for (int ks = 0; ks < S::K1S; ++ks)
                    z = M::mma(M::lds(x0 + (nt * 16 + lr) * S::P_IN + (ks * K + kq) * EB), w1[mt][ks], z);
#pragma unroll
                for (int i = 0; i < 4; ++i) t[mt][nt][i] = act_tanh(z[i]);
                g[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int ks = 0; ks < S::K2S; ++ks) {
                const Frag B_ = w2t(mt, ks);
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    g[nt] = M::mma(M::lds(dzs + (nt * 16 + lr) * S::P_H + (ks * K + kq) * EB), B_, g[nt]);
                // a few K-steps' operands in flight, not all (registers)
                if (ks % 4 == 3) __builtin_amdgcn_sched_barrier(0);
            }
            f32x4 dz1[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float th = t[mt][nt][i];
                    dz1[nt][i] = g[nt][i] * (1.0f - th * th);
                    db1a[mt] += dz1[nt][i];
                }
            // dW1 += dz1^T x0 (K = the tile's samples in accumulator order)
#pragma unroll
            for (int it = 0; it < S::KT; ++it) {
                if constexpr (DT == DT_BF16) {
                    dw1[mt][it] = M::mma(pack_acc_k(dz1[0], dz1[1]),
                                         lds_k_perm(x0T, S::P_T, it * 16 + lr, q), dw1[mt][it]);
                } else {
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float B_ = *reinterpret_cast<const float*>(
                                x0T + (it * 16 + lr) * S::P_T + (16 * nt + 4 * q + i) * EB);
                            dw1[mt][it] = M::mma(dz1[nt][i], B_, dw1[mt][it]);
                        }
                }
            }
        }
        // dW2 += dz2^T h1
        if constexpr (DT == DT_BF16) {
            Frag Bh[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) Bh[mt] = pack_acc_k(t[mt][0], t[mt][1]);
#pragma unroll
            for (int jt = 0; jt < NJT; ++jt) {
                const Frag A_ = lds_col_perm(dzs, S::P_H, jt * 16 + lr, q);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[jt][mt] = M::mma(A_, Bh[mt], acc[jt][mt]);
                if (jt % 4 == 3) __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float A_ = *reinterpret_cast<const float*>(
                            dzs + (16 * nt + 4 * q + i) * S::P_H + (jt * 16 + lr) * EB);
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[jt][mt] = M::mma(A_, t[mt][nt][i], acc[jt][mt]);
                    }
        }
    }
    float* out = a.part_bwd + (size_t)blockIdx.x * S::BWD_FLOATS;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int f0 = wave * S::FPW + mt * 16;
#pragma unroll
        for (int it = 0; it < S::KT; ++it)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (it * 16 + lr < KIN)
                    part_out(&out[(f0 + 4 * q + i) * KIN + it * 16 + lr], dw1[mt][it][i], a.accumulate);
        float v = db1a[mt];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (q == 0) part_out(&out[H * KIN + f0 + lr], v, a.accumulate);
    }
    float* w2o = a.part_w2 + (size_t)blockIdx.x * H * H;
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                part_out(&w2o[(size_t)(jt * 16 + 4 * q + i) * H + wave * S::FPW + mt * 16 + lr],
                         acc[jt][mt][i], a.accumulate);
}

// Reduction of the per-workgroup partial sums, one launch for every
// gradient tensor: segment y sums, for r < rows and c < cols,
// out[r][c] = sum over parts g of part[g * stride + off + r * cols_in + c], in a
// fixed order (eight contiguous groups of parts, each summed in order, then
// the groups in order).
struct SumSeg {
    const float* part;
    float* out;
    int64_t stride, off;
    int nparts, rows, cols, cols_in;
};
constexpr int kMaxSeg = 8;
struct SumTable {
    SumSeg seg[kMaxSeg];
};

// A workgroup takes 32 elements of a segment; the eight lanes of an element
// (one per 32-lane group) each sum a contiguous eighth of the parts in order,
// and the eight partial sums are added in group order: a fixed order, with
// eight times the loads in flight of one chain per element.
constexpr int kSumSplit = 8;
__global__ void __launch_bounds__(256) k_ac_sum(SumTable t) {
    __shared__ float red[kSumSplit][32];
    const SumSeg& sg = t.seg[blockIdx.y];
    const int el = threadIdx.x & 31, sub = threadIdx.x >> 5;
    const int64_t e = (int64_t)blockIdx.x * 32 + el;
    const bool ok = e < (int64_t)sg.rows * sg.cols;
    float s = 0.0f;
    if (ok) {
        const int r = (int)(e / sg.cols), c = (int)(e % sg.cols);
        const float* src = sg.part + sg.off + (int64_t)r * sg.cols_in + c;
        const int per = (sg.nparts + kSumSplit - 1) / kSumSplit;
        const int g0 = sub * per, g1 = min(sg.nparts, g0 + per);
        int g = g0;
        constexpr int kInFlight = 32;
        for (; g + kInFlight <= g1; g += kInFlight) {
            float v[kInFlight];
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) v[u] = src[(size_t)(g + u) * sg.stride];
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) s += v[u];
        }
        for (; g < g1; ++g) s += src[(size_t)g * sg.stride];
    }
    red[sub][el] = s;
    __syncthreads();
    if (ok && sub == 0) {
        float total = red[0][el];
#pragma unroll
        for (int k = 1; k < kSumSplit; ++k) total += red[k][el];
        sg.out[e] = total;
    }
}

// Adam (Kingma and Ba 2015, Algorithm 1) on element i; c1 and c2 are the bias
// corrections 1 - beta^t. The updated parameter is also stored in the
// policy's format (`store`, NULL to skip).
__device__ __forceinline__ void adam_elem(float* __restrict__ p, const float* __restrict__ g,
                                          float* __restrict__ m, float* __restrict__ v, int64_t i,
                                          float lr, float b1, float b2, float eps, float c1,
                                          float c2, void* __restrict__ store, int store_dtype) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (store) {
        if (store_dtype == DT_BF16)
            static_cast<__bf16*>(store)[i] = (__bf16)pi;
        else
            static_cast<float*>(store)[i] = pi;
    }
}

// One element per thread.
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
       float c2, void* __restrict__ store, int store_dtype) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) adam_elem(p, g, m, v, i, lr, b1, b2, eps, c1, c2, store, store_dtype);
}

// Several tensors in one launch: tensor blockIdx.y, the same element update.
__global__ void __launch_bounds__(256) k_adam_many(AdamTable t, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
    const AdamSeg& a = t.seg[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < a.n)
        adam_elem(a.param, a.grad, a.m, a.v, i, lr, b1, b2, eps, c1, c2, a.store, a.store_dtype);
}

template <int DT, int H, int KIN, int NHP>
struct AcVariant {
    using S = AcShape<DT, H, KIN, NHP>;
    // the two per-tile kernels over one chunk of samples
    static void chunk(const AcArgs& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_ac_fwd<DT, H, KIN, NHP>), dim3(grid), dim3(S::NTHR), 0, s, a);
        hipLaunchKernelGGL((k_ac_bwd<DT, H, KIN, NHP>), dim3(grid), dim3(S::NTHR), 0, s, a);
    }
    // the partial sums of every workgroup -> the gradients
    static hipError_t sum(const AcArgs& a, int grid, const AcOut& o, hipStream_t s) {
        const PolicyArgs& p = a.pol;
        const int F = S::FWD_FLOATS, B = S::BWD_FLOATS;
        SumTable t{};
        int ns = 0;
        int64_t most = 0;
        auto seg = [&](const float* part, int64_t stride, int nparts, int64_t off, int rows,
                       int cols, int cols_in, float* out) {
            t.seg[ns++] = SumSeg{part, out, stride, off, nparts, rows, cols, cols_in};
            most = std::max<int64_t>(most, (int64_t)rows * cols);
        };
        seg(a.part_fwd, F, grid, 0, p.n_head, H, H, o.w3);
        seg(a.part_fwd, F, grid, (int64_t)NHP * H, 1, H, H, o.b2);
        seg(a.part_fwd, F, grid, (int64_t)NHP * H + H, 1, p.n_head, p.n_head, o.b3);
        if (o.log_std) seg(a.part_fwd, F, grid, (int64_t)NHP * H + H + NHP, 1, 1, 1, o.log_std);
        seg(a.part_bwd, B, grid, 0, H, p.d_in, KIN, o.w1);
        seg(a.part_bwd, B, grid, (int64_t)H * KIN, 1, H, H, o.b1);
        seg(a.part_w2, (int64_t)H * H, grid, 0, H, H, H, o.w2);
        hipLaunchKernelGGL(k_ac_sum, dim3((unsigned)((most + 31) / 32), ns), dim3(256), 0, s, t);
        return hipGetLastError();
    }
    static size_t part_floats(int grid) {
        return (size_t)grid * (S::FWD_FLOATS + S::BWD_FLOATS + H * H);
    }
};

// (dtype, hidden, padded input width, padded head width) of the compiled
// update kernels: CartPole's FP32 policy, the BF16 policies with narrow and
// wide heads.
template <class F>
hipError_t with_variant(int dtype, int hidden, int d_in, int n_head, F&& f) {
    if (dtype == DT_F32 && hidden == 64 && d_in <= 4 && n_head <= 16)
        return f(AcVariant<DT_F32, 64, 4, 16>{});
    if (dtype == DT_BF16 && hidden == 256 && d_in <= 32 && n_head <= 16)
        return f(AcVariant<DT_BF16, 256, 32, 16>{});
    if (dtype == DT_BF16 && hidden == 256 && d_in <= 32 && n_head <= 64)
        return f(AcVariant<DT_BF16, 256, 32, 64>{});
    return hipErrorInvalidValue;
}

}  // namespace

bool ac_supported(int dtype, int hidden, int d_in, int n_head) {
    return with_variant(dtype, hidden, d_in, n_head, [](auto) { return hipSuccess; }) ==
           hipSuccess;
}

// Workspace: dz2 rows [n][H] and the partial sums; each part 256-byte
// aligned.
static size_t ac_round_up(size_t b) { return (b + 255) / 256 * 256; }

int64_t ac_chunk_samples(int64_t n) { return std::min<int64_t>(n, kAcChunk); }

// ------------------------------------------- allocation-free workspace --
// For callers that cannot allocate (graph capture, serving loops): the
// workspace of a gradient over at most kAcStaticSamples samples lives in a
// file-scope device array, one per GPU, for the life of the process. Its size
// is the largest workspace of the compiled update variants at that count
// (BF16 width 256 with the 64-wide head; every tile its own workgroup).
namespace {
constexpr size_t ac_round_up_c(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t ac_static_bytes() {
    constexpr size_t n = kAcStaticSamples, h = 256, eb = 2;
    constexpr size_t tiles = (n + kAcRows - 1) / kAcRows;
    constexpr size_t grid = tiles;   // ac_grid: min(tiles, CUs)
    constexpr size_t nhp = 64, kin = 32;
    constexpr size_t part = grid * ((nhp * h + h + nhp + 1) + (h * kin + h)) + grid * h * h;
    return 256 + ac_round_up_c(n * h * eb) + part * sizeof(float);
}
}  // namespace

static __device__ __align__(256) char scratch[ac_static_bytes()];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
static bool g_scratch_done[kMaxDevices];
static std::mutex g_scratch_mu;

size_t ac_static_capacity() { return ac_static_bytes(); }

// The current device's copy of the array (looked up once per device, with
// that device current); nullptr with the HIP error in *err on failure.
void* ac_static_workspace(hipError_t* err) {
    *err = hipSuccess;
    int dev = 0;
    if ((*err = hipGetDevice(&dev)) != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* ptr = nullptr;
        if ((*err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
        g_scratch_done[dev] = true;
    }
    return g_scratch_ptr[dev];
}

size_t ac_workspace_bytes(int dtype, int hidden, int64_t n, int grid) {
    n = ac_chunk_samples(n);
    const size_t eb = dtype == DT_BF16 ? 2 : 4;
    const size_t rows = (size_t)n * hidden * eb;
    // partial sums of the widest head compiled for this format and width
    size_t part = 0;
    if (dtype == DT_F32 && hidden == 64)
        part = AcVariant<DT_F32, 64, 4, 16>::part_floats(grid);
    else if (dtype == DT_BF16 && hidden == 256)
        part = AcVariant<DT_BF16, 256, 32, 64>::part_floats(grid);
    return 256 + ac_round_up(rows) + part * sizeof(float);
}

hipError_t launch_ac_grad(const AcLaunch& l, hipStream_t s) {
    const PolicyArgs& p = l.args.pol;
    return with_variant(l.dtype, p.hidden, p.d_in, p.n_head, [&](auto v) {
        using V = decltype(v);
        using S = typename V::S;
        const int64_t chunk = std::min<int64_t>(l.args.n, kAcChunk);
        const size_t eb = S::EB;
        const size_t rows = (size_t)chunk * p.hidden * eb;
        AcArgs a = l.args;
        char* w = reinterpret_cast<char*>(((uintptr_t)l.workspace + 255) / 256 * 256);
        a.dz2_rows = w;
        w += ac_round_up(rows);
        a.part_fwd = reinterpret_cast<float*>(w);
        a.part_bwd = a.part_fwd + (size_t)l.grid * S::FWD_FLOATS;
        a.part_w2 = a.part_bwd + (size_t)l.grid * S::BWD_FLOATS;
        // chunks of samples in stream order; inv_n stays 1 / (all samples)
        for (int64_t c0 = 0; c0 < l.args.n; c0 += chunk) {
            AcArgs c = a;
            c.n = std::min<int64_t>(chunk, l.args.n - c0);
            c.obs = l.args.obs + (size_t)c0 * p.d_in;
            c.action = static_cast<const char*>(l.args.action) + (size_t)c0 * (l.args.n_act ? 1 : 4);
            c.ret = l.args.ret + c0;
            c.adv = l.args.adv + c0;
            c.accumulate = c0 > 0;
            V::chunk(c, l.grid, s);
        }
        return V::sum(a, l.grid, l.out, s);
    });
}

hipError_t launch_adam_many(const AdamTable& t, int n_tensors, int64_t most, float lr, float b1,
                            float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam_many, dim3((unsigned)((most + 255) / 256), (unsigned)n_tensors),
                       dim3(256), 0, s, t, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, void* store,
                       int store_dtype, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n,
                       lr, b1, b2, eps, c1, c2, store, store_dtype);
    return hipGetLastError();
}

}  // namespace wsx
