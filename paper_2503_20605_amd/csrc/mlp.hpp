// gfx950 kernels of the learned warm start: a small fully connected network
// trained and evaluated with bf16 operands on the matrix cores (fp32
// accumulation), fp32 master weights, Adam.
//
//   k_gemm_bf16     C = A B with A, B bf16 (either operand k-contiguous or
//                   not), fp32 result: a 64x64 tile of C per workgroup, K in
//                   panels staged through LDS with 16-byte loads along the
//                   operand's contiguous index, the next panel fetched while
//                   the current one is multiplied, one 32x32 tile per
//                   wavefront through gfx950's v_mfma_f32_32x32x16_bf16;
//                   optional split of K over workgroups (fp32 atomic
//                   accumulation); epilogue: + bias, optional GELU (keeps
//                   the fp32 pre-activation and writes the bf16
//                   activation), or the GELU backward dZ = C * GELU'(Z)
//   k_mse_colsum    loss, dY = 2 (Y - T) / (B n) and the last layer's bias
//                   gradient (column sums of dY): 64 columns x 256 rows
//                   per workgroup, reduced in LDS, then added atomically
//   k_adam          Adam update of the fp32 master weights + bf16 copy
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lattice.hpp"

namespace iblb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMlpBlock = 256;  // 4 wavefronts, a 64x64 tile of C

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    const float cdf = 0.5f * (1.f + erff(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
    return cdf + z * pdf;
}

// C(i, j) = sum_k A(i, k) B(k, j) (+ bias[j]) with A, B bf16 and fp32
// accumulation.  Operand layouts (template arguments):
//   AT = 0: A(i, k) = A[i * lda + k]  (k contiguous);  AT = 1: A[k * lda + i]
//   BT = 0: B(k, j) = B[j * ldb + k]  (k contiguous);  BT = 1: B[k * ldb + j]
// A workgroup takes a 64x64 tile of C and walks K in panels of KP: every
// thread fetches its share of the next panel of both operands (KP / 32
// 16-byte pieces of eight elements along the operand's contiguous index)
// while the wavefronts multiply the current one out of LDS, where tiles are
// kept k-contiguous (rows of KP + 8 elements, so every lane's eight MFMA
// operands are one aligned 16-byte read).  avec / bvec = 0 fetches the
// pieces element by element (an operand whose contiguous extent or leading
// dimension is not a multiple of 8, or is not 16-byte aligned).  Elements
// outside M x N x [kbeg, kend) read as zero.
// Epilogue (act): 0: Cf = C + bias; 1: Cf = Z = C + bias, Hb = bf16(GELU(Z));
// 2: Cf = C * GELU'(Zpre), Hb = its bf16 copy (the backward of a GELU layer,
// Zpre its pre-activation, same layout as Hb; Cf may be null), and, when
// colsum is given, colsum[j] += the sum of column j over the rows (added
// atomically).  With gridDim.z = S > 1 the
// workgroups of z take k in [z kc, (z + 1) kc) and add their partial
// products to Cf atomically (Cf zeroed beforehand; no bias, act = 0).
//
// Operand and result layout of one 32x32x16 product (lane l of 64):
//   A: row l % 32, k = 8 (l / 32) + 0..7;  B: column l % 32, same k;
//   result register r: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Piece v (0 .. 64 KP / 8 - 1) of a 64 x KP panel of operand X whose rows r
// (i of A, j of B) start at rb and whose k start at k0.  T = 0: piece v
// holds row v / (KP / 8), k 8 (v % (KP / 8)) + 0..7; T = 1: k v / 8, rows
// 8 (v % 8) + 0..7.
template <int T, int KP>
__device__ __forceinline__ u32x4 panel_fetch(const uint16_t* __restrict__ X, long long ld, int R, int kend,
                                            int rb, int k0, int v, int vec) {
    int r, k;
    if (T == 0) {
        r = rb + v / (KP / 8);
        k = k0 + 8 * (v % (KP / 8));
    } else {
        k = k0 + v / 8;
        r = rb + 8 * (v % 8);
    }
    u32x4 out = {0u, 0u, 0u, 0u};
    if (vec) {
        // the contiguous extent is a multiple of 8: a piece lies wholly
        // inside or wholly outside
        if (r < R && k < kend)
            out = *reinterpret_cast<const u32x4*>(X + (T == 0 ? (long long)r * ld + k : (long long)k * ld + r));
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int ru = T == 0 ? r : r + u, ku = T == 0 ? k + u : k;
            const uint32_t e =
                (ru < R && ku < kend) ? X[T == 0 ? (long long)ru * ld + ku : (long long)ku * ld + ru] : 0u;
            out[u >> 1] |= e << (16 * (u & 1));
        }
    }
    return out;
}

// Piece v into the k-contiguous LDS tile S (rows of KP + 8 elements).
template <int T, int KP>
__device__ __forceinline__ void panel_stash(uint16_t* __restrict__ S, int v, u32x4 x) {
    constexpr int LD = KP + 8;
    if (T == 0) {
        *reinterpret_cast<u32x4*>(S + (v / (KP / 8)) * LD + 8 * (v % (KP / 8))) = x;
    } else {
        const int k = v / 8, r = 8 * (v % 8);
#pragma unroll
        for (int u = 0; u < 8; ++u) S[(r + u) * LD + k] = (uint16_t)(x[u >> 1] >> (16 * (u & 1)));
    }
}

template <int AT, int BT, int KP>
__global__ __launch_bounds__(kMlpBlock) void k_gemm_bf16(
    const uint16_t* __restrict__ A, long long lda, const uint16_t* __restrict__ B, long long ldb,
    float* __restrict__ Cf, uint16_t* __restrict__ Hb, long long ldc, const float* __restrict__ bias,
    const float* __restrict__ Zpre, float* __restrict__ colsum, int M, int N, int K, int act, int kc,
    int avec, int bvec) {
    constexpr int LD = KP + 8, NV = KP / 32;
    __shared__ __attribute__((aligned(16))) uint16_t As[64 * LD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * LD];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int ib = blockIdx.y * 64, jb = blockIdx.x * 64;
    const int kbeg = blockIdx.z * kc, kend = K < kbeg + kc ? K : kbeg + kc;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    u32x4 ra[NV], rb[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        ra[u] = panel_fetch<AT, KP>(A, lda, M, kend, ib, kbeg, t + kMlpBlock * u, avec);
        rb[u] = panel_fetch<BT, KP>(B, ldb, N, kend, jb, kbeg, t + kMlpBlock * u, bvec);
    }
    for (int k0 = kbeg; k0 < kend; k0 += KP) {
        if (k0 != kbeg) __syncthreads();  // the previous panel's reads are done
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            panel_stash<AT, KP>(As, t + kMlpBlock * u, ra[u]);
            panel_stash<BT, KP>(Bs, t + kMlpBlock * u, rb[u]);
        }
        __syncthreads();
        if (k0 + KP < kend) {
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                ra[u] = panel_fetch<AT, KP>(A, lda, M, kend, ib, k0 + KP, t + kMlpBlock * u, avec);
                rb[u] = panel_fetch<BT, KP>(B, ldb, N, kend, jb, k0 + KP, t + kMlpBlock * u, bvec);
            }
        }
        // k steps of 16 past kend hold zeros only: skipped
        const int nsteps = (kend - k0 < KP ? kend - k0 + 15 : KP) / 16;
#pragma unroll
        for (int s = 0; s < KP / 16; ++s) {
            if (s < nsteps) {
                const int kq = 16 * s + (lane >> 5) * 8;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(As + (wi + (lane & 31)) * LD + kq);
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bs + (wj + (lane & 31)) * LD + kq);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
        }
    }
    const int j = jb + wj + (lane & 31);
    if (j >= N) return;
    if (gridDim.z > 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = ib + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (i < M) unsafeAtomicAdd(Cf + (long long)i * ldc + j, acc[r]);
        }
        return;
    }
    const float bj = bias ? bias[j] : 0.f;
    float cs = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = ib + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i >= M) continue;
        const long long o = (long long)i * ldc + j;
        if (act == 2) {
            const float g = acc[r] * gelu_grad(Zpre[o]);
            if (Cf) Cf[o] = g;
            Hb[o] = f32_to_bf16_rne(g);
            cs += g;
        } else {
            const float z = acc[r] + bj;
            Cf[o] = z;
            if (act) Hb[o] = f32_to_bf16_rne(gelu(z));
        }
    }
    if (act == 2 && colsum) {
        // the column sums of dZ (the bias gradient of the layer below):
        // lanes l and l ^ 32 hold the two halves of column j's 32 rows
        cs += __shfl_xor(cs, 32, 64);
        if (lane < 32) unsafeAtomicAdd(colsum + j, cs);
    }
}

// The loss gradient of the last layer and its column sums: dY = 2 (Y - T) /
// (M N) for Y, T of M rows and N columns (row-major), written in bf16 for
// the products; colsum[j] += sum_i dY(i, j) (zeroed beforehand; the bias
// gradient); partial[block] = sum of (Y - T)^2 over the block's elements in
// fp64 (the loss, summed on the host in block order).  Workgroup (bx, by)
// takes 64 columns and rows [by kColsumRows, (by + 1) kColsumRows); its 16
// lane groups take every 16th row; the partial sums meet in LDS and each
// column's goes out with one atomic.
constexpr int kColsumBlock = 1024;
constexpr int kColsumRows = 256;
__global__ __launch_bounds__(kColsumBlock) void k_mse_colsum(const float* __restrict__ Y,
                                                              const float* __restrict__ T,
                                                              uint16_t* __restrict__ dYb,
                                                              float* __restrict__ colsum,
                                                              double* __restrict__ partial, int M, int N) {
    __shared__ float part[16][64];
    __shared__ double sq[16][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int i0 = blockIdx.y * kColsumRows, i1 = i0 + kColsumRows < M ? i0 + kColsumRows : M;
    const float scale = 2.f / (float)((long long)M * N);
    float s = 0.f;
    double e2 = 0.0;
    if (j < N)
        for (int i = i0 + g; i < i1; i += 16) {
            const long long o = (long long)i * N + j;
            const float e = Y[o] - T[o];
            const float d = scale * e;
            dYb[o] = f32_to_bf16_rne(d);
            s += d;
            e2 += (double)e * e;
        }
    part[g][c] = s;
    sq[g][c] = e2;
    __syncthreads();
    if (g == 0) {
        float t = 0.f;
        double q = 0.0;
        for (int k = 0; k < 16; ++k) {
            t += part[k][c];
            q += sq[k][c];
        }
        if (j < N) unsafeAtomicAdd(colsum + j, t);
        sq[0][c] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double q = 0.0;
        for (int k = 0; k < 64; ++k) q += sq[0][k];
        partial[blockIdx.y * gridDim.x + blockIdx.x] = q;
    }
}

// x[i] = 0 for i < n
__global__ void k_zero_f32(float* __restrict__ x, long long n) {
    const long long i = (long long)blockIdx.x * kMlpBlock + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

// Adam (Kingma & Ba) on the fp32 master copy; bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t.  Writes the bf16 copy used by the products.
__global__ void k_adam(float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                       float beta1, float beta2, float eps, float bc1, float bc2) {
    const long long i = (long long)blockIdx.x * kMlpBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    wb[i] = f32_to_bf16_rne(wi);
}

// fp32 -> bf16 (nearest even), n elements
__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * kMlpBlock + threadIdx.x;
    if (i < n) y[i] = f32_to_bf16_rne(x[i]);
}

}  // namespace iblb
