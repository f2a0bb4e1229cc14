// Surrogate MLP (protocol -> predicted fitness) with hand-written BF16 MFMA
// kernels: 128 -> 512 -> 512 -> 512 -> 1, GELU(x) = x Phi(x) on the hidden
// layers, BF16 weights and activations into v_mfma_f32_16x16x32_bf16 with FP32
// accumulation, FP32 master weights and Adam.  The surrogate only pre-screens
// GA offspring; the full simulation evaluates whatever it lets through.
//
// Net buffer (caller-owned, gga_mlp_net_bytes()):
//   header (normalisation mu, sigma) | params f32 | adam m | adam v | grads |
//   bf16 copies W_l [K][N] and W_l^T [N][K] for the three MFMA layers.
// Parameter order: W1 [128][512], b1, W2 [512][512], b2, W3 [512][512], b3,
// w4 [512], b4 [1].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "gga_device.h"
#include "gga_internal.h"
#include "mlp_internal.h"

namespace gga {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int PADK = 8;   // LDS rows of BK + PADK bf16 (the pad spreads banks)

// Phi(x), the standard normal CDF, through erf(|x| / sqrt 2) in the rational
// form of Abramowitz & Stegun 7.1.26 (Hastings): erf(a) = 1 - p(t) exp(-a^2),
// t = 1 / (1 + 0.3275911 a), |error| <= 1.5e-7, so Phi is within 7.5e-8 (plus
// fp32 rounding) everywhere.  Branch-free: one reciprocal and one exp2 against
// the two-branch polynomial of the library erff.  e receives exp(-x^2 / 2),
// which the derivative also needs.
__device__ __forceinline__ float phi_as(float x, float& e) {
    const float a = fabsf(x) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
    const float p =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
    e = __builtin_amdgcn_exp2f(-a * a * 1.4426950408889634f);
    return 0.5f + copysignf(0.5f * fmaf(-p, e, 1.0f), x);
}
// GELU(x) = x Phi(x) = relu(x) - |x| p(t) exp(-x^2 / 2) / 2 with the same
// rational erf (x Phi(x) = x/2 + |x| erf(|x| / sqrt 2) / 2): 11 VALU operations
// and two transcendentals, the 1/2 and 1/sqrt 2 folded into the constants.
// GELU'(x) = Phi(x) + x phi(x), phi(x) = exp(-x^2 / 2) / sqrt(2 pi).
__device__ __forceinline__ float gelu_f(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.2316418882f, ax, 1.0f));
    const float q =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 0.5307027145f, -0.7265760135f), 0.7107068705f), -0.142248368f),
                 0.127414796f);
    const float e = __builtin_amdgcn_exp2f(x * x * -0.7213475204f);
    return fmaf(-ax * q, e, fmaxf(x, 0.0f));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
    float e;
    const float p = phi_as(x, e);
    return fmaf(x * 0.39894228040143268f, e, p);
}

// One bf16x8 vector of an operand tile: elements (r, k0..k0+7) of a matrix
// X(r, k) = X[r*s_r + k*s_k] with `rows` x `K` bounds, zero outside.
__device__ __forceinline__ bf16x8 load8(const bf16* X, int s_r, int s_k, int rows, int K, int r, int k0) {
    bf16x8 v;
    if (s_k == 1 && r < rows && k0 + 8 <= K && ((s_r & 7) == 0)) {
        v = *reinterpret_cast<const bf16x8*>(X + (size_t)r * s_r + k0);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + e;
            v[e] = (r < rows && k < K) ? X[(size_t)r * s_r + (size_t)k * s_k] : (bf16)0.0f;
        }
    }
    return v;
}

// C = A (M x K) * B (K x N) with element A(m,k) = A[m*sa_m + k*sa_k] and
// B(k,n) = B[k*sb_k + n*sb_n].  256 threads (2 x 2 waves) compute a
// (32 WT) x (32 WT) tile, each wave WT x WT blocks of MFMA 16x16x32, over
// k-tiles of BK.  The operand tiles are double-buffered in LDS: the global
// loads of k-tile t + 1 are in flight while the MFMAs of k-tile t run.
template <int WT, int BK>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(MlpGemm g) {
    constexpr int TM = 32 * WT;                          // tile rows (= tile columns)
    constexpr int VPT = TM * BK / 8 / 256;               // bf16x8 vectors per thread per operand
    __shared__ bf16 As[2][TM][BK + PADK];
    __shared__ bf16 Bs[2][TM][BK + PADK];                // stored as [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TM / 2);
    floatx4 acc[WT][WT];
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ra[VPT], rb[VPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = tid + v * 256, r = idx / (BK / 8), k = (idx % (BK / 8)) * 8;
            ra[v] = load8(g.A, g.sa_m, g.sa_k, g.M, g.K, m0 + r, k0 + k);
            rb[v] = load8(g.B, g.sb_n, g.sb_k, g.N, g.K, n0 + r, k0 + k);   // B^T(n, k) = B(k, n)
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = tid + v * 256, r = idx / (BK / 8), k = (idx % (BK / 8)) * 8;
            *reinterpret_cast<bf16x8*>(&As[buf][r][k]) = ra[v];
            *reinterpret_cast<bf16x8*>(&Bs[buf][r][k]) = rb[v];
        }
    };
    const int nk = (g.K + BK - 1) / BK;
    fetch(0);
    stash(0);
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int t = 0; t < nk; ++t) {
        const int buf = t & 1;
        if (t + 1 < nk) fetch((t + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            bf16x8 b[WT];
#pragma unroll
            for (int j = 0; j < WT; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + j * 16 + fr][kk + fk]);
#pragma unroll
            for (int i = 0; i < WT; ++i) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[buf][wm + i * 16 + fr][kk + fk]);
#pragma unroll
                for (int j = 0; j < WT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
            }
        }
        if (t + 1 < nk) stash(buf ^ 1);                  // the other buffer: last read before the previous barrier
        __syncthreads();
    }
    // D[4*(lane/16) + r][lane%16] of every 16x16 block
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                float v = acc[i][j][r] + (g.bias ? g.bias[col] : 0.0f);
                if (g.mode == MLP_FWD || g.mode == MLP_INFER) {
                    if (g.mode == MLP_FWD) g.Z[(size_t)row * g.ldz + col] = v;
                    g.H[(size_t)row * g.ldh + col] = (bf16)gelu_f(v);
                } else if (g.mode == MLP_BWD) {
                    g.H[(size_t)row * g.ldh + col] = (bf16)(v * gelu_grad_f(g.Z[(size_t)row * g.ldz + col]));
                } else {
                    g.C[(size_t)row * g.ldc + col] = v;
                }
            }
}

// The same product when both operands run along K in memory (A [M][sa_m],
// B^T [N][sb_n]; every layer of the forward pass and the data gradient of the
// backward pass), K a multiple of 32 and N of the tile width: unguarded
// 16-byte loads (rows beyond M clamp to row M - 1 and are not stored), and the
// MFMA operands swapped so that each lane ends with four consecutive columns
// of one row, stored as one 16-byte (f32) or 8-byte (bf16) write.  The tile
// epilogue is fixed at compile time (MODE).  Workgroups are numbered so that
// the N / TM column tiles of one row block run on one XCD (blocks are dealt
// round-robin over the 8 XCDs), which then reads that row block once into its
// L2.  The accumulators start from the bias.  At most 122 VGPRs (no AGPRs),
// so four workgroups share a CU (their LDS tiles fill its 160 KB).  MLP_OUT (the last hidden layer of a prediction) stores no activations:
// it writes, per row and per chunk of TM / 2 columns, the partial dot product
// of the bf16-rounded GELU outputs with w4 into C[row][chunk].
template <int WT, int MODE>
__global__ __launch_bounds__(256, 2) void gemm_nt_kernel(MlpGemm g) {
    constexpr int TM = 32 * WT, BK = 32, VPT = TM * BK / 8 / 256, CPR = BK / 8;
    __shared__ bf16 As[2][TM][BK + PADK];
    __shared__ bf16 Bs[2][TM][BK + PADK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntn = g.N / TM;
    int bid = blockIdx.x;
    if ((gridDim.x & 7) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
    const int m0 = (bid / ntn) * TM, n0 = (bid - (bid / ntn) * ntn) * TM;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TM / 2);
    floatx4 acc[WT][WT];                                  // [column block][row block], from the bias
#pragma unroll
    for (int i = 0; i < WT; ++i) {
        floatx4 b0 = floatx4{0.f, 0.f, 0.f, 0.f};
        if (g.bias) {
            const float4 bb = *reinterpret_cast<const float4*>(g.bias + n0 + wn + i * 16 + (lane >> 4) * 4);
            b0 = floatx4{bb.x, bb.y, bb.z, bb.w};
        }
#pragma unroll
        for (int j = 0; j < WT; ++j) acc[i][j] = b0;
    }
    const bf16* pa[VPT];
    const bf16* pb[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
        const int idx = tid + v * 256, r = idx / CPR, k = (idx % CPR) * 8;
        pa[v] = g.A + (size_t)min(m0 + r, g.M - 1) * g.sa_m + k;
        pb[v] = g.B + (size_t)(n0 + r) * g.sb_n + k;
    }
    bf16x8 ra[VPT], rb[VPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            ra[v] = *reinterpret_cast<const bf16x8*>(pa[v] + k0);
            rb[v] = *reinterpret_cast<const bf16x8*>(pb[v] + k0);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = tid + v * 256, r = idx / CPR, k = (idx % CPR) * 8;
            *reinterpret_cast<bf16x8*>(&As[buf][r][k]) = ra[v];
            *reinterpret_cast<bf16x8*>(&Bs[buf][r][k]) = rb[v];
        }
    };
    const int nk = g.K / BK;
    fetch(0);
    stash(0);
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int t = 0; t < nk; ++t) {
        const int buf = t & 1;
        if (t + 1 < nk) fetch((t + 1) * BK);
        bf16x8 a[WT];
#pragma unroll
        for (int j = 0; j < WT; ++j) a[j] = *reinterpret_cast<const bf16x8*>(&As[buf][wm + j * 16 + fr][fk]);
#pragma unroll
        for (int i = 0; i < WT; ++i) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + i * 16 + fr][fk]);
#pragma unroll
            for (int j = 0; j < WT; ++j)                    // D^T block: rows n, columns m
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < nk) stash(buf ^ 1);
        __syncthreads();
    }
    typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
    // lane: row m0 + wm + 16 j + (lane & 15), columns n .. n + 3, n = n0 + wn + 16 i + 4 (lane >> 4)
#pragma unroll
    for (int j = 0; j < WT; ++j) {
        const int row = m0 + wm + j * 16 + (lane & 15);
        if (row >= g.M) continue;                         // the four lanes of a row share its fate
        float dot = 0.0f;
#pragma unroll
        for (int i = 0; i < WT; ++i) {
            const int col = n0 + wn + i * 16 + (lane >> 4) * 4;
            float o[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
            if (MODE == MLP_PLAIN) {
                *reinterpret_cast<float4*>(g.C + (size_t)row * g.ldc + col) = make_float4(o[0], o[1], o[2], o[3]);
                continue;
            }
            if (MODE == MLP_OUT) {                        // this lane's share of H3 . w4 (H3 rounded to bf16)
                const float4 w = *reinterpret_cast<const float4*>(g.w4 + col);
                dot = fmaf((float)(bf16)gelu_f(o[0]), w.x, dot);
                dot = fmaf((float)(bf16)gelu_f(o[1]), w.y, dot);
                dot = fmaf((float)(bf16)gelu_f(o[2]), w.z, dot);
                dot = fmaf((float)(bf16)gelu_f(o[3]), w.w, dot);
                continue;
            }
            if (MODE == MLP_FWD)
                *reinterpret_cast<float4*>(g.Z + (size_t)row * g.ldz + col) = make_float4(o[0], o[1], o[2], o[3]);
            if (MODE == MLP_BWD) {
                const float4 z = *reinterpret_cast<const float4*>(g.Z + (size_t)row * g.ldz + col);
                o[0] *= gelu_grad_f(z.x); o[1] *= gelu_grad_f(z.y); o[2] *= gelu_grad_f(z.z); o[3] *= gelu_grad_f(z.w);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) o[q] = gelu_f(o[q]);
            }
            bf16x4 h;
#pragma unroll
            for (int q = 0; q < 4; ++q) h[q] = (bf16)o[q];
            *reinterpret_cast<bf16x4*>(g.H + (size_t)row * g.ldh + col) = h;
        }
        if (MODE == MLP_OUT) {
            // lanes l, l + 16, l + 32, l + 48 hold one row: their sum is the
            // wave's partial over its TM / 2 columns, chunk (n0 + wn) / (TM / 2)
            dot += __shfl_xor(dot, 16, 64);
            dot += __shfl_xor(dot, 32, 64);
            if ((lane >> 4) == 0) g.C[(size_t)row * g.ldc + (n0 + wn) / (TM / 2)] = dot;
        }
    }
}

// C = A (M x K) * B (K x N) when both operands run along M and N in memory
// (A(m, k) = A[k sa_k + m], B(k, n) = B[k sb_k + n]: the weight gradients
// H^T dZ), over the k range [k0, k1) of split blockIdx.y, M and N multiples of
// the tile.  16-byte loads of 8 consecutive rows (or columns) at one k are
// transposed into the [row][k] LDS tiles the MFMA fragments read; rows of k
// past k1 load as zero.  Each split writes its own f32 slice C + split * ldp
// (a fixed-order sum over the splits follows when there are several).
template <int WT>
__global__ __launch_bounds__(256) void gemm_tn_kernel(MlpGemm g, int kchunk, long ldp) {
    constexpr int TM = 32 * WT, BK = 32, VPT = TM * BK / 8 / 256, VPR = TM / 8;
    __shared__ bf16 As[2][TM][BK + PADK];
    __shared__ bf16 Bs[2][TM][BK + PADK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntn = g.N / TM;
    const int m0 = (blockIdx.x / ntn) * TM, n0 = (blockIdx.x - (blockIdx.x / ntn) * ntn) * TM;
    const int kb = blockIdx.y * kchunk, ke = min(g.K, kb + kchunk);
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TM / 2);
    floatx4 acc[WT][WT];                                  // [column block][row block]
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ra[VPT], rb[VPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = tid + v * 256, k = k0 + idx / VPR, r = (idx % VPR) * 8;
            const bool in = k < ke;
            const bf16x8 z = {};
            ra[v] = in ? *reinterpret_cast<const bf16x8*>(g.A + (size_t)k * g.sa_k + m0 + r) : z;
            rb[v] = in ? *reinterpret_cast<const bf16x8*>(g.B + (size_t)k * g.sb_k + n0 + r) : z;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = tid + v * 256, k = idx / VPR, r = (idx % VPR) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                As[buf][r + e][k] = ra[v][e];
                Bs[buf][r + e][k] = rb[v][e];
            }
        }
    };
    const int nk = (ke - kb + BK - 1) / BK;
    if (nk > 0) {
        fetch(kb);
        stash(0);
    }
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int t = 0; t < nk; ++t) {
        const int buf = t & 1;
        if (t + 1 < nk) fetch(kb + (t + 1) * BK);
        bf16x8 a[WT];
#pragma unroll
        for (int j = 0; j < WT; ++j) a[j] = *reinterpret_cast<const bf16x8*>(&As[buf][wm + j * 16 + fr][fk]);
#pragma unroll
        for (int i = 0; i < WT; ++i) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + i * 16 + fr][fk]);
#pragma unroll
            for (int j = 0; j < WT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < nk) stash(buf ^ 1);
        __syncthreads();
    }
    float* C = g.C + (size_t)blockIdx.y * ldp;
#pragma unroll
    for (int j = 0; j < WT; ++j) {
        const int row = m0 + wm + j * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < WT; ++i) {
            const int col = n0 + wn + i * 16 + (lane >> 4) * 4;
            *reinterpret_cast<float4*>(C + (size_t)row * g.ldc + col) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
    }
}

// out[i] = sum over splits s = 0 .. S-1 (in order) of part[s * n + i], 4 per thread
__global__ void split_sum_kernel(const float* part, int S, long n, float* out) {
    const long i = ((long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i >= n) return;
    float4 acc = *reinterpret_cast<const float4*>(part + i);
    for (int s = 1; s < S; ++s) {
        const float4 v = *reinterpret_cast<const float4*>(part + (size_t)s * n + i);
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    *reinterpret_cast<float4*>(out + i) = acc;
}

// Features of protocol b: for fraction j < 40, (dose/5, gap/60, 1) if present.
// One thread per 8 consecutive features (fractions j0 .. j0 + 3), stored as one
// 16-byte vector; the dose and delay loads depend only on K, so they are in
// flight together with the load of nfrac[b].
__global__ void encode_kernel(const float* dose, const int32_t* gap, const int32_t* nfrac, int B, int K,
                              bf16* X) {
    constexpr int V = MLP_IN / 8;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * V) return;
    const int b = idx / V, f0 = (idx - b * V) * 8, j0 = f0 / 3;
    const int jmax = min(MLP_FRAC, K);
    float d[4], g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool in = j0 + q < jmax;
        d[q] = in ? dose[(size_t)b * K + j0 + q] * (1.0f / 5.0f) : 0.0f;
        g[q] = in ? (float)gap[(size_t)b * K + j0 + q] * (1.0f / 60.0f) : 0.0f;
    }
    const int nf = min(jmax, nfrac[b]);
    bf16x8 x;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int f = f0 + e, j = f / 3, part = f - 3 * j, q = j - j0;
        const float v = part == 0 ? d[q] : part == 1 ? g[q] : 1.0f;
        x[e] = (bf16)(j < nf ? v : 0.0f);
    }
    *reinterpret_cast<bf16x8*>(X + (size_t)b * MLP_IN + f0) = x;
}

// y[b] = H3[b] . w4 + b4 (one wave per sample); optionally de-normalised.
__global__ void out_fwd_kernel(const bf16* H3, const float* w4, const float* b4, int B, float* y,
                               const float* norm) {
    const int b = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= B) return;
    float s = 0.0f;
    for (int k = lane; k < MLP_HID; k += 64) s += (float)H3[(size_t)b * MLP_HID + k] * w4[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[b] = norm ? (s + b4[0]) * norm[1] + norm[0] : s + b4[0];
}

// y[b] = sum over chunks c (in order) of part[b][c] + b4; optionally de-normalised.
__global__ void out_sum_kernel(const float* part, int nchunk, int ld, const float* b4, int B, float* y,
                               const float* norm) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)b * ld + c];
    y[b] = norm ? (s + b4[0]) * norm[1] + norm[0] : s + b4[0];
}

// dy = 2 (y - t') / B with t' = (t - mu) / sigma; loss = mean (y - t')^2.
__global__ __launch_bounds__(256) void loss_kernel(const float* y, const float* t, const float* norm, int B,
                                                   float* dy, float* loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const float e = y[b] - (t[b] - norm[0]) / norm[1];
        dy[b] = 2.0f * e / (float)B;
        s += e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = red[0] / (float)B;
}

// dZ3[b][k] = dy[b] w4[k] gelu'(Z3[b][k])
__global__ void out_bwd_kernel(const float* dy, const float* w4, const float* Z3, int B, bf16* dZ3) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * MLP_HID) return;
    const int b = idx / MLP_HID, k = idx - b * MLP_HID;
    dZ3[idx] = (bf16)(dy[b] * w4[k] * gelu_grad_f(Z3[idx]));
}

// Column sums of a [B][N] bf16 matrix (bias gradients), and dw4 / db4.
// Column sums over the batch, in two deterministic passes: block c adds the
// rows of chunk c, each lane 8 consecutive columns (one 16-byte load per row)
// in 4 row groups of one wave each, combined in LDS in a fixed order; the
// final pass adds the chunks in order.  Row b is weighted by w[b] when w is
// given, and column N then holds the sum of w.  N <= 512, N % 8 == 0.
__global__ __launch_bounds__(256) void colsum_partial_kernel(const bf16* D, const float* w, int B, int N,
                                                             float* part) {
    __shared__ float red[4][MLP_HID];
    __shared__ float redw[4];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6, c = blockIdx.x;
    const int col = lane * 8;
    const int rows = (B + MLP_RED_CHUNKS - 1) / MLP_RED_CHUNKS;
    const int b0 = c * rows, b1 = min(B, b0 + rows);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float sw = 0.0f;
    for (int b = b0 + grp; b < b1; b += 4) {
        const float wb = w ? w[b] : 1.0f;
        if (col < N) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(D + (size_t)b * N + col);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += (float)v[e] * wb;
        }
        sw += wb;
    }
    if (col < N) {
#pragma unroll
        for (int e = 0; e < 8; ++e) red[grp][col + e] = s[e];
    }
    if (lane == 0) redw[grp] = sw;
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += blockDim.x)
        part[(size_t)c * (N + 1) + n] = ((red[0][n] + red[1][n]) + red[2][n]) + red[3][n];
    if (w && threadIdx.x == 0) part[(size_t)c * (N + 1) + N] = ((redw[0] + redw[1]) + redw[2]) + redw[3];
}
__global__ void colsum_final_kernel(const float* part, int N, int with_w, float* out, float* out_w) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n > N || (n == N && !with_w)) return;
    float s = 0.0f;
    for (int c = 0; c < MLP_RED_CHUNKS; ++c) s += part[(size_t)c * (N + 1) + n];
    if (n < N) out[n] = s;
    else out_w[0] = s;
}

// Adam with bias correction over the flat parameter vector.
__global__ void adam_kernel(float* p, float* m, float* v, const float* g, long n, float lr, const int32_t* step) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float t = (float)*step;                       // bias corrections of step t
    const float c1 = 1.0f - powf(0.9f, t), c2 = 1.0f - powf(0.999f, t);
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// bf16 copies W [K][N] and W^T [N][K] of a K x N layer.
__global__ void refresh_kernel(const float* W, int K, int N, bf16* Wb, bf16* WTb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * N) return;
    const int k = idx / N, n = idx - k * N;
    const bf16 v = (bf16)W[idx];
    Wb[idx] = v;
    WTb[(size_t)n * K + k] = v;
}

// Weights uniform on +-1/sqrt(fan_in) from Philox blocks (i, 0x4D4C5000, layer, 0);
// biases and Adam state zero.
__global__ void init_kernel(float* p, float* m, float* v, float* g, long n, uint32_t k0, uint32_t k1) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long off = i;
    int layer = -1;
    float fan_in = 1.0f;
    const long sizes[8] = {(long)MLP_IN * MLP_HID, MLP_HID, (long)MLP_HID * MLP_HID, MLP_HID,
                           (long)MLP_HID * MLP_HID, MLP_HID, MLP_HID, 1};
    const float fans[8] = {(float)MLP_IN, 0.f, (float)MLP_HID, 0.f, (float)MLP_HID, 0.f, (float)MLP_HID, 0.f};
    for (int t = 0; t < 8; ++t) {
        if (off < sizes[t]) { layer = t; fan_in = fans[t]; break; }
        off -= sizes[t];
    }
    float w = 0.0f;
    if (fan_in > 0.0f) {
        const Block4 b = philox10((uint32_t)i, 0x4D4C5000u, (uint32_t)layer, 0u, k0, k1);
        const float u = ((float)(b.w0 >> 8) + 0.5f) * (1.0f / 16777216.0f);
        w = (2.0f * u - 1.0f) / sqrtf(fan_in);
    }
    p[i] = w;
    m[i] = 0.0f;
    v[i] = 0.0f;
    g[i] = 0.0f;
}

// mu, sigma of n targets (one block, float64 accumulation).
__global__ __launch_bounds__(256) void norm_kernel(const float* t, int n, float* norm) {
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) { a += t[i]; b += (double)t[i] * t[i]; }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) { s1[threadIdx.x] += s1[threadIdx.x + w]; s2[threadIdx.x] += s2[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = n ? s1[0] / n : 0.0;
        const double var = n ? s2[0] / n - mu * mu : 1.0;
        norm[0] = (float)mu;
        norm[1] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
    }
}

unsigned blocks_for(long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

namespace {
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Operands that run along K, K a multiple of 32, N of the tile width, and
// 16-byte alignment of every row the epilogue and the loads touch.
bool nt_eligible(const MlpGemm& g, int TM) {
    if (g.sa_k != 1 || g.sb_k != 1 || g.K <= 0 || g.K % 32 || g.N % TM) return false;
    if (g.sa_m % 8 || g.sb_n % 8 || !aligned16(g.A) || !aligned16(g.B)) return false;
    if (g.bias && !aligned16(g.bias)) return false;
    if (g.mode == MLP_PLAIN) return aligned16(g.C) && g.ldc % 4 == 0;
    if (g.mode == MLP_OUT) return g.C && g.w4 && aligned16(g.w4) && g.ldc >= g.N / (TM / 2);
    if (g.mode != MLP_INFER && (!aligned16(g.Z) || g.ldz % 4)) return false;
    return aligned16(g.H) && g.ldh % 4 == 0;
}

template <int WT>
void launch_nt(const MlpGemm& g, hipStream_t s) {
    const dim3 grid(blocks_for(g.M, 32 * WT) * (g.N / (32 * WT)));
    switch (g.mode) {
        case MLP_FWD: hipLaunchKernelGGL((gemm_nt_kernel<WT, MLP_FWD>), grid, dim3(256), 0, s, g); break;
        case MLP_INFER: hipLaunchKernelGGL((gemm_nt_kernel<WT, MLP_INFER>), grid, dim3(256), 0, s, g); break;
        case MLP_BWD: hipLaunchKernelGGL((gemm_nt_kernel<WT, MLP_BWD>), grid, dim3(256), 0, s, g); break;
        case MLP_OUT: hipLaunchKernelGGL((gemm_nt_kernel<WT, MLP_OUT>), grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL((gemm_nt_kernel<WT, MLP_PLAIN>), grid, dim3(256), 0, s, g); break;
    }
}
}  // namespace

// Both operands along M and N, M and N multiples of 64, 16-byte aligned rows.
bool tn_eligible(const MlpGemm& g) {
    if (g.mode != MLP_PLAIN || g.sa_m != 1 || g.sb_n != 1 || g.K <= 0 || g.M % 64 || g.N % 64) return false;
    if (g.sa_k % 8 || g.sb_k % 8 || !aligned16(g.A) || !aligned16(g.B) || g.bias) return false;
    return aligned16(g.C) && g.ldc % 4 == 0;
}

// 128 x 128 tiles when they still give the chip two workgroups per CU, else 64 x 64
int gemm_tile(const MlpGemm& g) { return (long)blocks_for(g.N, 128) * blocks_for(g.M, 128) >= 512 ? 128 : 64; }

hipError_t launch_gemm(const MlpGemm& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const bool large = gemm_tile(g) == 128;
    if (nt_eligible(g, large ? 128 : 64)) {
        if (large) launch_nt<4>(g, s);
        else launch_nt<2>(g, s);
        return hipGetLastError();
    }
    if (g.mode == MLP_OUT) return hipErrorInvalidValue;    // only the K-contiguous kernel fuses the output layer
    if (tn_eligible(g)) {
        hipLaunchKernelGGL((gemm_tn_kernel<2>), dim3((g.M / 64) * (g.N / 64), 1), dim3(256), 0, s, g, g.K, 0L);
        return hipGetLastError();
    }
    if (large)
        hipLaunchKernelGGL((gemm_bf16_kernel<4, 32>), dim3(blocks_for(g.N, 128), blocks_for(g.M, 128)), dim3(256), 0, s,
                           g);
    else
        hipLaunchKernelGGL((gemm_bf16_kernel<2, 32>), dim3(blocks_for(g.N, 64), blocks_for(g.M, 64)), dim3(256), 0, s,
                           g);
    return hipGetLastError();
}

hipError_t mlp_forward(const MlpNet& net, const float* dose, const int32_t* gap, const int32_t* nfrac, int B,
                       int K, const MlpWork& w, float* pred, bool predict, hipStream_t s) {
    hipLaunchKernelGGL(encode_kernel, dim3(blocks_for((long)B * (MLP_IN / 8), 256)), dim3(256), 0, s, dose, gap,
                       nfrac, B, K, w.X);
    hipError_t e = hipGetLastError();
    const bf16* in = w.X;
    int kin = MLP_IN, nchunk = 0;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        MlpGemm g{};
        g.M = B; g.N = MLP_HID; g.K = kin;
        g.A = in; g.sa_m = kin; g.sa_k = 1;
        g.B = net.WT[l]; g.sb_k = 1; g.sb_n = kin;           // B(k, n) = W^T[n][k]
        g.bias = net.b[l];
        g.mode = predict ? MLP_INFER : MLP_FWD;          // a prediction keeps no pre-activations
        g.Z = w.Z[l]; g.ldz = MLP_HID;
        g.H = w.H[l]; g.ldh = MLP_HID;
        if (predict && l == 2) {                          // output layer fused: partial dot products in Z[0]
            g.mode = MLP_OUT;
            g.w4 = net.w4;
            g.C = w.Z[0]; g.ldc = 16;
            nchunk = MLP_HID / (gemm_tile(g) / 2);
        }
        e = launch_gemm(g, s);
        in = w.H[l];
        kin = MLP_HID;
    }
    if (e != hipSuccess) return e;
    if (predict)
        hipLaunchKernelGGL(out_sum_kernel, dim3(blocks_for(B, 256)), dim3(256), 0, s, w.Z[0], nchunk, 16, net.b4, B,
                           pred, net.norm);
    else
        hipLaunchKernelGGL(out_fwd_kernel, dim3(blocks_for(B, 4)), dim3(256), 0, s, w.H[2], net.w4, net.b4, B, pred,
                           nullptr);
    return hipGetLastError();
}

// A weight gradient (K = batch rows): K split over S workgroups per tile so
// that the 16-64 tiles of a 512-wide layer fill the chip, S = B / 512 up to 8,
// partials in `part` (part_floats >= S M N; the caller's spent Z3 buffer),
// then summed in split order.
hipError_t launch_wgrad(const MlpGemm& g, float* part, long part_floats, hipStream_t s) {
    if (!tn_eligible(g)) return launch_gemm(g, s);
    const long mn = (long)g.M * g.N;
    int S = std::min(8, std::max(1, g.K / 512));
    while (S > 1 && (long)S * mn > part_floats) --S;
    const int kchunk = ((g.K + S - 1) / S + 31) / 32 * 32;
    S = (g.K + kchunk - 1) / kchunk;
    MlpGemm p = g;
    if (S > 1) { p.C = part; p.ldc = g.N; }
    hipLaunchKernelGGL((gemm_tn_kernel<2>), dim3((g.M / 64) * (g.N / 64), S), dim3(256), 0, s, p, kchunk, mn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    hipLaunchKernelGGL(split_sum_kernel, dim3(blocks_for(mn / 4, 256)), dim3(256), 0, s, part, S, mn, g.C);
    return hipGetLastError();
}

hipError_t mlp_backward(const MlpNet& net, int B, const float* target, const MlpWork& w, float* loss,
                        hipStream_t s) {
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, w.y, target, net.norm, B, w.dy, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // dw4 = H3^T dy, db4 = sum dy
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(MLP_RED_CHUNKS), dim3(256), 0, s, w.H[2], w.dy, B,
                       MLP_HID, w.part);
    hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks_for(MLP_HID + 1, 256)), dim3(256), 0, s, w.part, MLP_HID, 1,
                       net.gw4, net.gb4);
    hipLaunchKernelGGL(out_bwd_kernel, dim3(blocks_for((long)B * MLP_HID, 256)), dim3(256), 0, s, w.dy, net.w4,
                       w.Z[2], B, w.dZ[0]);
    e = hipGetLastError();
    // layer l = 2, 1, 0: dZ_l in dZ[cur]; weight and bias gradients, then dZ_{l-1}
    int cur = 0;
    for (int l = 2; l >= 0 && e == hipSuccess; --l) {
        const bf16* hin = l == 0 ? w.X : w.H[l - 1];
        const int kin = l == 0 ? MLP_IN : MLP_HID;
        MlpGemm g{};
        g.M = kin; g.N = MLP_HID; g.K = B;                    // dW_l = H_in^T dZ_l
        g.A = hin; g.sa_m = 1; g.sa_k = kin;
        g.B = w.dZ[cur]; g.sb_k = MLP_HID; g.sb_n = 1;
        g.mode = MLP_PLAIN;
        g.C = net.gW[l]; g.ldc = MLP_HID;
        e = launch_wgrad(g, w.Z[2], (long)B * MLP_HID, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(colsum_partial_kernel, dim3(MLP_RED_CHUNKS), dim3(256), 0, s, w.dZ[cur],
                           nullptr, B, MLP_HID, w.part);
        hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks_for(MLP_HID, 256)), dim3(256), 0, s, w.part, MLP_HID, 0,
                           net.gb[l], nullptr);
        e = hipGetLastError();
        if (l == 0 || e != hipSuccess) break;
        MlpGemm d{};
        d.M = B; d.N = MLP_HID; d.K = MLP_HID;                // dZ_{l-1} = (dZ_l W_l^T) . gelu'(Z_{l-1})
        d.A = w.dZ[cur]; d.sa_m = MLP_HID; d.sa_k = 1;
        d.B = net.W[l]; d.sb_k = 1; d.sb_n = MLP_HID;         // B(k, n) = W_l[n][k]
        d.mode = MLP_BWD;
        d.Z = w.Z[l - 1]; d.ldz = MLP_HID;
        d.H = w.dZ[1 - cur]; d.ldh = MLP_HID;
        e = launch_gemm(d, s);
        cur = 1 - cur;
    }
    return e;
}

hipError_t mlp_adam_refresh(const MlpNet& net, int step, float lr, hipStream_t s) {
    const long n = MLP_PARAMS;
    // the net's step counter: set to `step`, or advanced by one when step is 0
    hipError_t e = launch_counter(net.step, step > 0 ? step : 1, step > 0 ? 0 : 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, net.p, net.m, net.v, net.g, n, lr,
                       net.step);
    e = hipGetLastError();
    for (int l = 0; l < 3 && e == hipSuccess; ++l) e = mlp_refresh_layer(net, l, s);
    return e;
}

hipError_t mlp_refresh_layer(const MlpNet& net, int l, hipStream_t s) {
    const int K = l == 0 ? MLP_IN : MLP_HID;
    hipLaunchKernelGGL(refresh_kernel, dim3(blocks_for((long)K * MLP_HID, 256)), dim3(256), 0, s, net.Wf[l], K,
                       MLP_HID, net.W[l], net.WT[l]);
    return hipGetLastError();
}

hipError_t mlp_init(const MlpNet& net, uint64_t seed, hipStream_t s) {
    const long n = MLP_PARAMS;
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, net.p, net.m, net.v, net.g, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    hipError_t e = hipGetLastError();
    for (int l = 0; l < 3 && e == hipSuccess; ++l) e = mlp_refresh_layer(net, l, s);
    return e;
}

hipError_t mlp_set_norm(const MlpNet& net, const float* t, int n, hipStream_t s) {
    hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(256), 0, s, t, n, net.norm);
    return hipGetLastError();
}

}  // namespace gga
