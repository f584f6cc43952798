// gfx950 kernels of the learned warm start: a small fully connected network
// trained and evaluated with bf16 operands on the matrix cores (fp32
// accumulation), fp32 master weights, Adam.
//
//   k_gemm_bf16     C = A B with A, B bf16 in any strides, fp32 result: a
//                   64x64 tile of C per workgroup, operands staged through
//                   LDS 32 k at a time (loads along whichever index is
//                   contiguous), one 32x32 tile per wavefront through
//                   gfx950's v_mfma_f32_32x32x16_bf16; optional split of K over
//                   workgroups (fp32 atomic accumulation); epilogue: + bias,
//                   optional GELU (keeps the fp32 pre-activation and writes
//                   the bf16 activation)
//   k_gelu_back     dZ = dH * GELU'(Z), bf16 copy for the next products
//   k_colsum        bias gradient (column sums of dZ): 64 columns x 256
//                   rows per workgroup, reduced in LDS, then added
//                   atomically
//   k_mse           loss and dY = 2 (Y - T) / (B n)
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

// C(i, j) = sum_k A(i, k) B(k, j) (+ bias[j]); A(i, k) = A[i * sai + k * sak],
// B(k, j) = B[k * sbk + j * sbj].  act = 0: C fp32 to Cf[i * ldc + j];
// act = 1: Cf gets the pre-activation and Hb[i * ldc + j] the bf16 GELU.
// Operands outside M x N x K read as zero.  With gridDim.z = S > 1 the
// workgroups of z take the k range [z kc, (z + 1) kc) and add their partial
// products to Cf atomically (Cf zeroed beforehand; no bias, act = 0).
//
// Operand and result layout of one 32x32x16 product (lane l of 64):
//   A: row l % 32, k = 8 (l / 32) + 0..7;  B: column l % 32, same k;
//   result register r: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
constexpr int kGemmK = 32;         // k per LDS stage
constexpr int kGemmLd = kGemmK + 8;  // padded LDS row (bf16 elements; 80 bytes, so
                                     // each lane's 8 operands are one aligned 16-byte read)

__global__ __launch_bounds__(kMlpBlock) void k_gemm_bf16(
    const uint16_t* __restrict__ A, long long sai, long long sak, const uint16_t* __restrict__ B,
    long long sbk, long long sbj, float* __restrict__ Cf, uint16_t* __restrict__ Hb, long long ldc,
    const float* __restrict__ bias, int M, int N, int K, int act, int kc) {
    // tiles stored k-contiguous: As[i][k], Bs[j][k]
    __shared__ __attribute__((aligned(16))) uint16_t As[64 * kGemmLd];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * kGemmLd];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int ib = blockIdx.y * 64, jb = blockIdx.x * 64;
    const int kbeg = blockIdx.z * kc, kend = K < kbeg + kc ? K : kbeg + kc;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    // each thread stages 8 elements of each operand per stage, along the
    // operand's contiguous index so that neighbouring threads read
    // neighbouring addresses
    const bool a_kc = sak == 1, b_kc = sbk == 1;
    for (int k0 = kbeg; k0 < kend; k0 += kGemmK) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            int ii, kk;
            if (a_kc) {  // k contiguous: thread -> row t / 4, 8 consecutive k
                ii = t >> 2;
                kk = (t & 3) * 8 + u;
            } else {     // i contiguous: thread -> k t / 8, 8 consecutive rows
                kk = t >> 3;
                ii = (t & 7) * 8 + u;
            }
            const int gi = ib + ii, gk = k0 + kk;
            As[ii * kGemmLd + kk] = (gi < M && gk < kend) ? A[gi * sai + gk * sak] : (uint16_t)0;
            int jj;
            if (b_kc) {
                jj = t >> 2;
                kk = (t & 3) * 8 + u;
            } else {
                kk = t >> 3;
                jj = (t & 7) * 8 + u;
            }
            const int gj = jb + jj, gk2 = k0 + kk;
            Bs[jj * kGemmLd + kk] = (gj < N && gk2 < kend) ? B[gk2 * sbk + gj * sbj] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int s16 = 0; s16 < kGemmK; s16 += 16) {
            const int kq = s16 + (lane >> 5) * 8;
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(As + (wi + (lane & 31)) * kGemmLd + kq);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bs + (wj + (lane & 31)) * kGemmLd + kq);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int j = jb + wj + (lane & 31);
    if (j >= N) return;
    if (gridDim.z > 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = ib + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (i < M) unsafeAtomicAdd(Cf + i * ldc + j, acc[r]);
        }
        return;
    }
    const float bj = bias ? bias[j] : 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = ib + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i >= M) continue;
        const float z = acc[r] + bj;
        Cf[i * ldc + j] = z;
        if (act) Hb[i * ldc + j] = f32_to_bf16_rne(gelu(z));
    }
}

// dZ = dH * GELU'(Z) (fp32 and bf16 copies), n elements
__global__ void k_gelu_back(const float* __restrict__ dH, const float* __restrict__ Z,
                            float* __restrict__ dZf, uint16_t* __restrict__ dZb, long long n) {
    const long long i = (long long)blockIdx.x * kMlpBlock + threadIdx.x;
    if (i >= n) return;
    const float g = dH[i] * gelu_grad(Z[i]);
    dZf[i] = g;
    dZb[i] = f32_to_bf16_rne(g);
}

// out[j] += sum_i X[i * N + j] (out zeroed beforehand): workgroup
// (bx, by) takes 64 columns and rows [by kColsumRows, (by + 1) kColsumRows);
// its 16 lane groups sum every 16th row, the 16 partial sums are added in
// LDS and the result atomically to out.
constexpr int kColsumBlock = 1024;
constexpr int kColsumRows = 256;
__global__ __launch_bounds__(kColsumBlock) void k_colsum(const float* __restrict__ X,
                                                          float* __restrict__ out, int M, int N) {
    __shared__ float part[16][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int i0 = blockIdx.y * kColsumRows, i1 = i0 + kColsumRows < M ? i0 + kColsumRows : M;
    float s = 0.f;
    if (j < N)
        for (int i = i0 + g; i < i1; i += 16) s += X[(long long)i * N + j];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && j < N) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += part[k][c];
        unsafeAtomicAdd(out + j, t);
    }
}

// x[i] = 0 for i < n
__global__ void k_zero_f32(float* __restrict__ x, long long n) {
    const long long i = (long long)blockIdx.x * kMlpBlock + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

// dY = 2 (Y - T) / n (fp32 and bf16), per-block partial sums of (Y - T)^2
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                      float* __restrict__ dYf, uint16_t* __restrict__ dYb,
                      double* __restrict__ partial, long long n) {
    __shared__ double sh[kMlpBlock];
    const long long i = (long long)blockIdx.x * kMlpBlock + threadIdx.x;
    double e2 = 0.0;
    if (i < n) {
        const float e = Y[i] - T[i];
        const float g = 2.f * e / (float)n;
        dYf[i] = g;
        dYb[i] = f32_to_bf16_rne(g);
        e2 = (double)e * e;
    }
    sh[threadIdx.x] = e2;
    __syncthreads();
    for (int o = kMlpBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
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
