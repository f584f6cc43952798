// Host runtime and C ABI of the warm-start network (see iblb.h): a fully
// connected network widths[0] -> ... -> widths[L] with GELU after every
// layer but the last, bf16 operands on the matrix cores, fp32 master
// weights, MSE loss, Adam.  All device memory comes from the caller's
// workspace, except the static scratch array of the forward pass that
// allocates nothing (iblb_mlp_forward_noalloc).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#pragma GCC visibility push(default)
#include "iblb.h"
#pragma GCC visibility pop
#include "mlp.hpp"

using namespace iblb;

// Scratch of iblb_mlp_forward_noalloc: the input rounded to bf16 and the
// hidden layers' activations, for callers that cannot allocate device
// memory.  Each device holds its own copy for the life of the process;
// every such call on a device shares it.
constexpr size_t kNoallocScratchBytes = 8u << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr size_t kMlpAlign = 256;
size_t mlp_align(size_t v) { return (v + kMlpAlign - 1) / kMlpAlign * kMlpAlign; }
long long mlp_cdiv(long long a, long long b) { return (a + b - 1) / b; }

struct MlpLayout {
    int L = 0, B = 0, maxw = 0;
    std::vector<int> w;
    std::vector<long long> woff, boff;  // offsets in the packed parameter vector
    long long P = 0;
    size_t master, grad, m, v, wb, xb, partial, total;
    size_t dZb[2];  // output-side gradients (bf16) of two consecutive layers, used in turn
    std::vector<size_t> Z, H;  // Z[l]: layer l output (fp32); H[l]: layer l input (bf16)
};

bool mlp_plan(int L, const int* widths, int B, MlpLayout& Y, std::string& err) {
    if (L < 1 || L > 16 || !widths) { err = "n_layers must be 1..16 with widths given"; return false; }
    if (B < 1) { err = "max_batch must be >= 1"; return false; }
    Y.L = L;
    Y.B = B;
    Y.w.assign(widths, widths + L + 1);
    Y.maxw = 0;
    for (int x : Y.w) {
        if (x < 1 || x > 65536) { err = "layer widths must be 1..65536"; return false; }
        Y.maxw = std::max(Y.maxw, x);
    }
    Y.woff.resize(L);
    Y.boff.resize(L);
    Y.P = 0;
    for (int l = 0; l < L; ++l) {
        Y.woff[l] = Y.P;
        Y.P += (long long)Y.w[l] * Y.w[l + 1];
        Y.boff[l] = Y.P;
        Y.P += Y.w[l + 1];
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = mlp_align(o + bytes); return at; };
    Y.master = take(4 * Y.P);
    Y.grad = take(4 * Y.P);
    Y.m = take(4 * Y.P);
    Y.v = take(4 * Y.P);
    Y.wb = take(2 * Y.P);
    Y.Z.resize(L);
    Y.H.resize(L);
    for (int l = 0; l < L; ++l) {
        Y.Z[l] = take(4ull * B * Y.w[l + 1]);
        Y.H[l] = take(2ull * B * Y.w[l]);
    }
    Y.xb = Y.H[0];
    for (int h = 0; h < 2; ++h) Y.dZb[h] = take(2ull * B * Y.maxw);
    Y.partial = take(8ull * mlp_cdiv(Y.w[L], 64) * mlp_cdiv(B, kColsumRows));
    Y.total = o;
    return true;
}

}  // namespace

struct iblb_mlp {
    MlpLayout Y;
    char* ws = nullptr;
    char* scratch = nullptr;  // device address of this device's static scratch
    hipStream_t stream = nullptr;
    long long t = 0;       // Adam steps taken
    int last_batch = 0;    // batch of the last gradient evaluation
    std::string err;
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

thread_local std::string g_mlp_err;

int mlp_fail(iblb_mlp* c, int code, const std::string& msg) {
    if (c) c->err = msg; else g_mlp_err = msg;
    return code;
}

#define MLPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return mlp_fail(ctx, IBLB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// One operand of a product: its elements, leading dimension and layout
// (t = 0: k contiguous, t = 1: the row / column index contiguous).
struct Operand {
    const uint16_t* p;
    long long ld;
    int t;
};

// 16-byte pieces need a contiguous extent and leading dimension that are
// multiples of 8 elements and a 16-byte aligned base.
int pieces_ok(const Operand& X, int ext) {
    return X.ld % 8 == 0 && ext % 8 == 0 && (reinterpret_cast<uintptr_t>(X.p) & 15) == 0;
}

template <int KP>
void launch_gemm(const iblb_mlp* c, dim3 grid, const Operand& A, const Operand& B, float* Cf, uint16_t* Hb,
                 long long ldc, const float* bias, const float* Zpre, float* colsum, int M, int N, int K, int act,
                 int kc,
                 int avec, int bvec) {
    const dim3 block(kMlpBlock);
    const int sel = 2 * A.t + B.t;
    if (sel == 0)
        hipLaunchKernelGGL((k_gemm_bf16<0, 0, KP>), grid, block, 0, c->stream, A.p, A.ld, B.p, B.ld, Cf, Hb,
                           ldc, bias, Zpre, colsum, M, N, K, act, kc, avec, bvec);
    else if (sel == 1)
        hipLaunchKernelGGL((k_gemm_bf16<0, 1, KP>), grid, block, 0, c->stream, A.p, A.ld, B.p, B.ld, Cf, Hb,
                           ldc, bias, Zpre, colsum, M, N, K, act, kc, avec, bvec);
    else if (sel == 2)
        hipLaunchKernelGGL((k_gemm_bf16<1, 0, KP>), grid, block, 0, c->stream, A.p, A.ld, B.p, B.ld, Cf, Hb,
                           ldc, bias, Zpre, colsum, M, N, K, act, kc, avec, bvec);
    else
        hipLaunchKernelGGL((k_gemm_bf16<1, 1, KP>), grid, block, 0, c->stream, A.p, A.ld, B.p, B.ld, Cf, Hb,
                           ldc, bias, Zpre, colsum, M, N, K, act, kc, avec, bvec);
}

// C (M x N, leading dimension ldc) = A B.  With split_k, K is divided over
// enough workgroups to give the device about 1024 of them (at most 16
// pieces, each a multiple of the LDS panel); the pieces add into Cf, which
// the caller has zeroed.  Only plain products (no bias, act 0) split.
// Panels of 128 k: against 256-k panels (one fetch for K = 256, half the
// workgroups per compute unit) and splits aiming at 256 workgroups, the
// training step of the 4-256-256-256-1280 network on 4096 samples took
// 0.297 against 0.313 ms.
void gemm(const iblb_mlp* c, const Operand& A, const Operand& B, float* Cf, uint16_t* Hb, long long ldc,
          const float* bias, const float* Zpre, int M, int N, int K, int act, bool split_k = false,
          float* colsum = nullptr) {
    constexpr int KP = 128;
    const long long tiles = mlp_cdiv(N, 64) * mlp_cdiv(M, 64);
    int splits = 1;
    if (split_k && !bias && act == 0) {
        const long long want = mlp_cdiv(1024, tiles);
        splits = (int)std::max(1LL, std::min({want, 16LL, mlp_cdiv(K, KP)}));
    }
    const int kc = (int)(mlp_cdiv(mlp_cdiv(K, splits), KP) * KP);
    splits = (int)mlp_cdiv(K, kc);
    const int avec = pieces_ok(A, A.t == 0 ? K : M), bvec = pieces_ok(B, B.t == 0 ? K : N);
    const dim3 grid((unsigned)mlp_cdiv(N, 64), (unsigned)mlp_cdiv(M, 64), (unsigned)splits);
    launch_gemm<KP>(c, grid, A, B, Cf, Hb, ldc, bias, Zpre, colsum, M, N, K, act, kc, avec, bvec);
}

// forward pass of `batch` rows from device fp32 input x
int mlp_forward(iblb_mlp* c, const float* d_x, int batch) {
    const MlpLayout& Y = c->Y;
    const long long nx = (long long)batch * Y.w[0];
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)mlp_cdiv(nx, kMlpBlock)), dim3(kMlpBlock), 0, c->stream,
                       d_x, c->at<uint16_t>(Y.xb), nx);
    for (int l = 0; l < Y.L; ++l) {
        const int in = Y.w[l], out = Y.w[l + 1];
        const bool act = l < Y.L - 1;
        // Z = H W + b: H (batch x in) k-contiguous, W (in x out) row-major
        gemm(c, {c->at<uint16_t>(Y.H[l]), in, 0}, {c->at<uint16_t>(Y.wb) + Y.woff[l], out, 1},
             c->at<float>(Y.Z[l]), act ? c->at<uint16_t>(Y.H[l + 1]) : nullptr, out,
             c->at<float>(Y.master) + Y.boff[l], nullptr, batch, out, in, act ? 1 : 0);
    }
    MLPCHK(c, hipGetLastError());
    return IBLB_OK;
}

// Device address of the static scratch array on the current device, looked
// up once per device (host code must never pass the array's own name to a
// kernel: on the host that name is a stand-in, not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

hipError_t scratch_address(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Bytes of static scratch a forward pass of `batch` rows needs: the bf16
// input, one fp32 pre-activation buffer and two bf16 activation buffers of
// the widest hidden layer (the last layer writes the caller's output).
size_t noalloc_bytes(const MlpLayout& Y, long long batch) {
    int mh = 0;
    for (int l = 1; l < Y.L; ++l) mh = std::max(mh, Y.w[l]);
    size_t need = mlp_align(2ull * batch * Y.w[0]);
    if (mh > 0) need += mlp_align(4ull * batch * mh) + 2 * mlp_align(2ull * batch * mh);
    return need;
}

int check_batch(iblb_mlp* c, int batch) {
    if (!c) return IBLB_EINVAL;
    if (batch < 1 || batch > c->Y.B) return mlp_fail(c, IBLB_EINVAL, "batch must be 1..max_batch");
    return IBLB_OK;
}

}  // namespace

extern "C" {

size_t iblb_mlp_workspace_bytes(int n_layers, const int* widths, int max_batch) {
    MlpLayout Y;
    std::string err;
    return mlp_plan(n_layers, widths, max_batch, Y, err) ? Y.total : 0;
}

int iblb_mlp_create(int n_layers, const int* widths, int max_batch, void* d_ws, size_t ws_bytes,
                    void* stream, iblb_mlp** out) {
    if (!out) return mlp_fail(nullptr, IBLB_EINVAL, "out must not be NULL");
    *out = nullptr;
    MlpLayout Y;
    std::string err;
    if (!mlp_plan(n_layers, widths, max_batch, Y, err)) return mlp_fail(nullptr, IBLB_EINVAL, err);
    if (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % kMlpAlign)
        return mlp_fail(nullptr, IBLB_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < Y.total) return mlp_fail(nullptr, IBLB_ENOMEM, "workspace too small");
    char* scr = nullptr;
    hipError_t e = scratch_address(&scr);
    if (e != hipSuccess) {
        g_mlp_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return IBLB_EDEVICE;
    }
    iblb_mlp* c = new iblb_mlp();
    c->Y = Y;
    c->ws = static_cast<char*>(d_ws);
    c->scratch = scr;
    c->stream = static_cast<hipStream_t>(stream);
    e = hipMemsetAsync(c->ws, 0, Y.total, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_mlp_err = std::string("hipMemsetAsync: ") + hipGetErrorString(e);
        delete c;
        return IBLB_EDEVICE;
    }
    *out = c;
    return IBLB_OK;
}

int iblb_mlp_destroy(iblb_mlp* c) {
    delete c;
    return IBLB_OK;
}

const char* iblb_mlp_last_error(const iblb_mlp* c) { return c ? c->err.c_str() : g_mlp_err.c_str(); }

long long iblb_mlp_param_count(const iblb_mlp* c) { return c ? c->Y.P : 0; }

int iblb_mlp_set_params(iblb_mlp* c, const float* h_params) {
    if (!c) return IBLB_EINVAL;
    if (!h_params) return mlp_fail(c, IBLB_EINVAL, "NULL parameters");
    const MlpLayout& Y = c->Y;
    std::vector<float> tmp(h_params, h_params + Y.P);
    MLPCHK(c, hipMemcpyAsync(c->at<float>(Y.master), tmp.data(), 4 * Y.P, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipMemsetAsync(c->at<float>(Y.m), 0, 4 * Y.P, c->stream));
    MLPCHK(c, hipMemsetAsync(c->at<float>(Y.v), 0, 4 * Y.P, c->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)mlp_cdiv(Y.P, kMlpBlock)), dim3(kMlpBlock), 0, c->stream,
                       (const float*)c->at<float>(Y.master), c->at<uint16_t>(Y.wb), Y.P);
    MLPCHK(c, hipGetLastError());
    MLPCHK(c, hipStreamSynchronize(c->stream));
    c->t = 0;
    return IBLB_OK;
}

int iblb_mlp_get_params(iblb_mlp* c, float* h_params) {
    if (!c) return IBLB_EINVAL;
    if (!h_params) return mlp_fail(c, IBLB_EINVAL, "NULL parameters");
    MLPCHK(c, hipMemcpyAsync(h_params, c->at<float>(c->Y.master), 4 * c->Y.P, hipMemcpyDeviceToHost,
                             c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return IBLB_OK;
}

int iblb_mlp_forward(iblb_mlp* c, const float* d_x, int batch, float* d_y) {
    int rc = check_batch(c, batch);
    if (rc) return rc;
    if (!d_x || !d_y) return mlp_fail(c, IBLB_EINVAL, "NULL input or output");
    if ((rc = mlp_forward(c, d_x, batch))) return rc;
    const MlpLayout& Y = c->Y;
    MLPCHK(c, hipMemcpyAsync(d_y, c->at<float>(Y.Z[Y.L - 1]), 4ull * batch * Y.w[Y.L],
                             hipMemcpyDeviceToDevice, c->stream));
    return IBLB_OK;
}

int iblb_mlp_forward_noalloc(iblb_mlp* c, const float* d_x, int batch, float* d_y) {
    if (!c) return IBLB_EINVAL;
    if (batch < 1) return mlp_fail(c, IBLB_EINVAL, "batch must be >= 1");
    if (!d_x || !d_y) return mlp_fail(c, IBLB_EINVAL, "NULL input or output");
    const MlpLayout& Y = c->Y;
    const size_t need = noalloc_bytes(Y, batch);
    if (need > kNoallocScratchBytes) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "forward_noalloc: a batch of %d rows needs %zu bytes of static scratch, more than "
                 "its %zu",
                 batch, need, kNoallocScratchBytes);
        return mlp_fail(c, IBLB_EINVAL, buf);
    }
    // carve the scratch: bf16 input, fp32 pre-activations, two bf16
    // activation buffers used in turn (no clearing needed: every kernel
    // writes each element it later reads)
    int mh = 0;
    for (int l = 1; l < Y.L; ++l) mh = std::max(mh, Y.w[l]);
    char* p = c->scratch;
    uint16_t* xb = reinterpret_cast<uint16_t*>(p);
    p += mlp_align(2ull * batch * Y.w[0]);
    float* z = reinterpret_cast<float*>(p);
    p += mlp_align(4ull * batch * mh);
    uint16_t* h[2] = {reinterpret_cast<uint16_t*>(p),
                      reinterpret_cast<uint16_t*>(p + mlp_align(2ull * batch * mh))};
    const long long nx = (long long)batch * Y.w[0];
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)mlp_cdiv(nx, kMlpBlock)), dim3(kMlpBlock), 0, c->stream,
                       d_x, xb, nx);
    const uint16_t* in_b = xb;
    for (int l = 0; l < Y.L; ++l) {
        const int in = Y.w[l], out = Y.w[l + 1];
        const bool last = l == Y.L - 1;
        uint16_t* hb = last ? nullptr : h[l & 1];
        gemm(c, {in_b, in, 0}, {c->at<uint16_t>(Y.wb) + Y.woff[l], out, 1}, last ? d_y : z, hb, out,
             c->at<float>(Y.master) + Y.boff[l], nullptr, batch, out, in, last ? 0 : 1);
        in_b = hb;
    }
    MLPCHK(c, hipGetLastError());
    return IBLB_OK;
}

int iblb_mlp_gradients(iblb_mlp* c, const float* d_x, const float* d_t, int batch, float* h_grads,
                       double* loss) {
    int rc = check_batch(c, batch);
    if (rc) return rc;
    if (!d_x || !d_t) return mlp_fail(c, IBLB_EINVAL, "NULL input or target");
    if ((rc = mlp_forward(c, d_x, batch))) return rc;
    const MlpLayout& Y = c->Y;
    const int L = Y.L;
    const long long ny = (long long)batch * Y.w[L];
    const dim3 lgrid((unsigned)mlp_cdiv(Y.w[L], 64), (unsigned)mlp_cdiv(batch, kColsumRows));
    const int nblk = (int)(lgrid.x * lgrid.y);
    float* grad = c->at<float>(Y.grad);
    // the gradients of every layer are accumulated atomically: zeroed first
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)mlp_cdiv(Y.P, kMlpBlock)), dim3(kMlpBlock), 0, c->stream, grad,
                       Y.P);
    // dZ of layer l lives in buffer (L - 1 - l) % 2; the loss gradient also
    // gives the last layer's bias gradient
    hipLaunchKernelGGL(k_mse_colsum, lgrid, dim3(kColsumBlock), 0, c->stream,
                       (const float*)c->at<float>(Y.Z[L - 1]), d_t, c->at<uint16_t>(Y.dZb[0]),
                       grad + Y.boff[L - 1], c->at<double>(Y.partial), batch, Y.w[L]);
    for (int l = L - 1; l >= 0; --l) {
        const int in = Y.w[l], out = Y.w[l + 1];
        const int h = (L - 1 - l) & 1;
        const uint16_t* dZb = c->at<uint16_t>(Y.dZb[h]);
        // bias: the column sums of dZ, formed with dZ itself (k_mse_colsum,
        // or the epilogue of the product that forms it); weights: H^T dZ
        // (K = batch, split over workgroups); input side: dZ W^T, times
        // GELU'(Z) of the layer below
        gemm(c, {c->at<uint16_t>(Y.H[l]), in, 1}, {dZb, out, 1}, grad + Y.woff[l], nullptr, out, nullptr, nullptr,
             in, out, batch, 0, true);
        if (l > 0)
            // (dZ of the layer below is needed in bf16 only: its column sums
            // are formed here)
            gemm(c, {dZb, out, 0}, {c->at<uint16_t>(Y.wb) + Y.woff[l], out, 0}, nullptr,
                 c->at<uint16_t>(Y.dZb[h ^ 1]), in, nullptr, c->at<float>(Y.Z[l - 1]), batch, in, out, 2, false,
                 grad + Y.boff[l - 1]);
    }
    MLPCHK(c, hipGetLastError());
    c->last_batch = batch;
    if (loss) {
        std::vector<double> part(nblk);
        MLPCHK(c, hipMemcpyAsync(part.data(), c->at<double>(Y.partial), 8ull * nblk, hipMemcpyDeviceToHost,
                                 c->stream));
        MLPCHK(c, hipStreamSynchronize(c->stream));
        double s = 0.0;
        for (double x : part) s += x;
        *loss = s / (double)ny;
    }
    if (h_grads) {
        MLPCHK(c, hipMemcpyAsync(h_grads, grad, 4 * Y.P, hipMemcpyDeviceToHost, c->stream));
        MLPCHK(c, hipStreamSynchronize(c->stream));
    }
    return IBLB_OK;
}

int iblb_mlp_adam_step(iblb_mlp* c, float lr, float beta1, float beta2, float eps) {
    if (!c) return IBLB_EINVAL;
    if (c->last_batch == 0) return mlp_fail(c, IBLB_EINVAL, "no gradients yet");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return mlp_fail(c, IBLB_EINVAL, "bad Adam hyper-parameters");
    const MlpLayout& Y = c->Y;
    c->t += 1;
    const float bc1 = 1.f - powf(beta1, (float)c->t), bc2 = 1.f - powf(beta2, (float)c->t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)mlp_cdiv(Y.P, kMlpBlock)), dim3(kMlpBlock), 0, c->stream,
                       c->at<float>(Y.master), c->at<uint16_t>(Y.wb), (const float*)c->at<float>(Y.grad),
                       c->at<float>(Y.m), c->at<float>(Y.v), Y.P, lr, beta1, beta2, eps, bc1, bc2);
    MLPCHK(c, hipGetLastError());
    return IBLB_OK;
}

}  // extern "C"
