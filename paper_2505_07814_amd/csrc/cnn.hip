// cnn.hip - C ABI of the learned initial guess (include/ptyr_cnn.h): launches
// of the BF16 matrix-core convolution kernels of cnn.hpp for inference,
// training gradients, Adam and patch stitching.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "cnn.hpp"
#include "ptyr_cnn.h"

using namespace ptyr::cnn;

struct ptyr_cnn {
    int B_max;
    char* ws;
    hipStream_t stream;
    size_t X[NLAYER], G[NLAYER], out, wbf, wt, wpart, lpart, loss, err, total;
};

namespace {

constexpr int LOSS_BLOCKS = 256;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t wpart_floats(int B) {
    size_t m = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const size_t nchunk = ((size_t)B * HOUT[l] * HOUT[l] + WCHUNK - 1) / WCHUNK;
        const size_t f = nchunk * (w_size(l) + COUTP[l]);
        if (f > m) m = f;
    }
    return m;
}

// workspace offsets for batches of up to B neighbourhoods
void layout(ptyr_cnn* c, int B) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int l = 0; l < NLAYER; ++l) c->X[l] = take((size_t)B * act_elems(l) * 2);
    for (int l = 0; l < NLAYER; ++l) c->G[l] = take((size_t)B * grad_elems(l) * 2);
    c->out = take((size_t)B * OUT * OUT * 4);
    c->wbf = take((size_t)NPARAM * 2);
    c->wt = take((size_t)WT_TOTAL * 2);
    c->wpart = take(wpart_floats(B) * 4);
    c->lpart = take(LOSS_BLOCKS * 8);
    c->loss = take(8);
    c->err = take(4);
    c->total = off;
}

template <class T>
T* at(ptyr_cnn* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

int blocks_for(size_t n, int per = 256) {
    size_t b = (n + per - 1) / per;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

ptyr_status launched() { return hipGetLastError() == hipSuccess ? PTYR_OK : PTYR_E_DEVICE; }

template <int L>
void fwd_layer(ptyr_cnn* c, const float* params, int B, float* out) {
    const int nblk = (B * HOUT[L] * HOUT[L] + 63) / 64;
    __bf16* Y = L < NLAYER - 1 ? at<__bf16>(c, c->X[L + 1]) : nullptr;
    hipLaunchKernelGGL(k_fwd<L>, dim3(nblk), dim3(256), 0, c->stream, at<__bf16>(c, c->X[L]),
                       at<__bf16>(c, c->wbf) + w_off(L), params + b_off(L), Y, out, B);
}

template <int L>
void bwd_layer(ptyr_cnn* c, int B, float* grad) {
    constexpr int NT = kp(L) / 16, PW = w_size(L) + COUTP[L];
    const int nchunk = (B * HOUT[L] * HOUT[L] + WCHUNK - 1) / WCHUNK;
    hipLaunchKernelGGL(k_wgrad<L>, dim3(nchunk, (NT + wg_nt<L>() - 1) / wg_nt<L>()), dim3(256), 0, c->stream,
                       at<__bf16>(c, c->G[L]), at<__bf16>(c, c->X[L]), at<float>(c, c->wpart), B);
    // weights and bias are contiguous in the parameter vector: one reduction
    hipLaunchKernelGGL(k_wreduce, dim3((PW + 31) / 32), dim3(256), 0, c->stream, at<float>(c, c->wpart), nchunk, PW,
                       grad + w_off(L));
    if constexpr (L > 0) {
        const int nblk = (B * HIN[L] * HIN[L] + 63) / 64;
        hipLaunchKernelGGL(k_dgrad<L>, dim3(nblk), dim3(256), 0, c->stream, at<__bf16>(c, c->G[L]),
                           at<__bf16>(c, c->wt) + wt_off(L), at<__bf16>(c, c->X[L]), at<__bf16>(c, c->G[L - 1]), B);
    }
}

// weights to BF16, gathered log input, the five layers; output to `out`
void run_forward(ptyr_cnn* c, const float* params, const float* pat, int n_pat, const int* nbr, int B, float* out) {
    const int nprep = NPARAM > WT_TOTAL ? NPARAM : WT_TOTAL;
    hipLaunchKernelGGL(k_prep, dim3((nprep + 255) / 256), dim3(256), 0, c->stream, params, at<__bf16>(c, c->wbf),
                       at<__bf16>(c, c->wt));
    hipLaunchKernelGGL(k_input, dim3(blocks_for((size_t)B * IN * IN)), dim3(256), 0, c->stream, pat, n_pat, nbr, B,
                       at<__bf16>(c, c->X[0]), at<int>(c, c->err));
    fwd_layer<0>(c, params, B, nullptr);
    fwd_layer<1>(c, params, B, nullptr);
    fwd_layer<2>(c, params, B, nullptr);
    fwd_layer<3>(c, params, B, nullptr);
    fwd_layer<4>(c, params, B, out);
}

ptyr_status check_batch(ptyr_cnn* c, const float* params, const float* pat, int n_pat, const int* nbr, int B) {
    if (!c || !params || !pat || !nbr) return PTYR_E_ARG;
    if (B < 1 || B > c->B_max || n_pat < 1) return PTYR_E_ARG;
    return PTYR_OK;
}

}  // namespace

extern "C" {

size_t ptyr_cnn_param_count(void) { return (size_t)NPARAM; }

size_t ptyr_cnn_workspace_bytes(int B_max) {
    if (B_max < 1) return 0;
    ptyr_cnn c;
    layout(&c, B_max);
    return c.total;
}

ptyr_status ptyr_cnn_create(int B_max, void* workspace, size_t ws_bytes, void* stream, ptyr_cnn** out) {
    if (!out) return PTYR_E_ARG;
    *out = nullptr;
    if (B_max < 1 || !workspace) return PTYR_E_ARG;
    ptyr_cnn* c = new (std::nothrow) ptyr_cnn;
    if (!c) return PTYR_E_NOMEM;
    c->B_max = B_max;
    c->ws = static_cast<char*>(workspace);
    c->stream = static_cast<hipStream_t>(stream);
    layout(c, B_max);
    if (ws_bytes < c->total) {
        delete c;
        return PTYR_E_NOMEM;
    }
    if (hipMemsetAsync(at<int>(c, c->err), 0, sizeof(int), c->stream) != hipSuccess) {
        delete c;
        return PTYR_E_DEVICE;
    }
    *out = c;
    return PTYR_OK;
}

void ptyr_cnn_destroy(ptyr_cnn* ctx) { delete ctx; }

ptyr_status ptyr_cnn_sync(ptyr_cnn* c) {
    if (!c) return PTYR_E_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return PTYR_E_DEVICE;
    int e = 0;
    if (hipMemcpy(&e, at<int>(c, c->err), sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return PTYR_E_DEVICE;
    if (e) {
        const int z = 0;
        if (hipMemcpy(at<int>(c, c->err), &z, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return PTYR_E_DEVICE;
        return PTYR_E_ARG;
    }
    return PTYR_OK;
}

ptyr_status ptyr_cnn_forward(ptyr_cnn* c, const float* params, const float* patterns, int n_pat, const int* nbr,
                             int B, float* out) {
    ptyr_status st = check_batch(c, params, patterns, n_pat, nbr, B);
    if (st != PTYR_OK) return st;
    if (!out) return PTYR_E_ARG;
    run_forward(c, params, patterns, n_pat, nbr, B, out);
    return launched();
}

ptyr_status ptyr_cnn_gradient(ptyr_cnn* c, const float* params, const float* patterns, int n_pat, const int* nbr,
                              const float* target, int B, float* grad, double* loss_dev) {
    ptyr_status st = check_batch(c, params, patterns, n_pat, nbr, B);
    if (st != PTYR_OK) return st;
    if (!target || !grad) return PTYR_E_ARG;
    float* out = at<float>(c, c->out);
    run_forward(c, params, patterns, n_pat, nbr, B, out);
    const int n = B * OUT * OUT;
    const int nblk = blocks_for(n) < LOSS_BLOCKS ? blocks_for(n) : LOSS_BLOCKS;
    hipLaunchKernelGGL(k_mse_partial, dim3(nblk), dim3(256), 0, c->stream, out, target, n, at<double>(c, c->lpart));
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, c->stream, at<double>(c, c->lpart), nblk, n,
                       loss_dev ? loss_dev : at<double>(c, c->loss));
    hipLaunchKernelGGL(k_mse_grad, dim3(blocks_for(n)), dim3(256), 0, c->stream, out, target, n,
                       at<__bf16>(c, c->G[NLAYER - 1]));
    bwd_layer<4>(c, B, grad);
    bwd_layer<3>(c, B, grad);
    bwd_layer<2>(c, B, grad);
    bwd_layer<1>(c, B, grad);
    bwd_layer<0>(c, B, grad);
    return launched();
}

ptyr_status ptyr_cnn_adam(ptyr_cnn* c, float* params, const float* grad, float* m, float* v, int64_t step, float lr,
                          float beta1, float beta2, float eps) {
    if (!c || !params || !grad || !m || !v || step < 1) return PTYR_E_ARG;
    const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(NPARAM)), dim3(256), 0, c->stream, params, grad, m, v, NPARAM, lr, beta1,
                       beta2, eps, (float)bc1, (float)std::sqrt(bc2));
    return launched();
}

ptyr_status ptyr_cnn_stitch(ptyr_cnn* c, const float* patches, const float* centres, int P, int H, int W, float* img) {
    if (!c || !img || H < 1 || W < 1 || P < 0) return PTYR_E_ARG;
    if (P > 0 && (!patches || !centres)) return PTYR_E_ARG;
    hipLaunchKernelGGL(k_stitch, dim3(blocks_for((size_t)H * W)), dim3(256), 0, c->stream, patches, centres, P, H, W,
                       img);
    return launched();
}

}  // extern "C"
