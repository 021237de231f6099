// cnn.hpp - kernels of the learned initial guess: a 5-layer 3x3 convolutional
// net that maps the log diffraction patterns of a 3 x 3 scan neighbourhood
// (9 x 64 x 64) to the projected phase of the 32 x 32 patch centred on the
// middle position.
//
//   layer  in          out         stride   reduction K = 9 taps x Cin (padded)
//   0      9(16) x 64  32 x 64     1        144 -> 160
//   1      32 x 64     32 x 32     2        288
//   2      32 x 32     32 x 32     1        288
//   3      32 x 32     32 x 32     1        288
//   4      32 x 32     1(16) x 32  1        288        (no ReLU after it)
//
// Every convolution and both of its gradients is an implicit GEMM on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation).  Activations and back-propagated gradients are stored NHWC in
// BF16 with channels padded to 16 / 32, so the 8 consecutive reduction elements
// a lane feeds to the MFMA are 8 consecutive channels of one pixel: one
// 16-byte load.  Lane i of a wave holds A[i%16][8(i/16)..+7],
// B[8(i/16)..+7][i%16] and receives D[4(i/16)..+3][i%16].
//
// Parameters are one FP32 vector: per layer W[Cout_p][K_p] with reduction
// index k = (3 u + v) * Cin_p + c for tap (u, v) and input channel c (padding
// entries are zero and stay zero under training, their gradient being exactly
// zero), followed by bias[Cout_p].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptyr {
namespace cnn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float floatx4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

constexpr int NLAYER = 5;
constexpr int NB = 9;             // patterns per neighbourhood
constexpr int IN = 64;            // pattern side
constexpr int OUT = 32;           // phase patch side
constexpr int CIN[NLAYER] = {9, 32, 32, 32, 32};
constexpr int CINP[NLAYER] = {16, 32, 32, 32, 32};
constexpr int COUT[NLAYER] = {32, 32, 32, 32, 1};
constexpr int COUTP[NLAYER] = {32, 32, 32, 32, 16};
constexpr int STRIDE[NLAYER] = {1, 2, 1, 1, 1};
constexpr int HIN[NLAYER] = {64, 64, 32, 32, 32};
constexpr int HOUT[NLAYER] = {64, 32, 32, 32, 32};

constexpr int pad32(int x) { return (x + 31) / 32 * 32; }
constexpr int kp(int l) { return pad32(9 * CINP[l]); }          // forward / weight-gradient reduction
constexpr int kd(int l) { return pad32(9 * COUTP[l]); }         // input-gradient reduction
constexpr int w_size(int l) { return COUTP[l] * kp(l); }
constexpr int w_off(int l) { return l == 0 ? 0 : w_off(l - 1) + w_size(l - 1) + COUTP[l - 1]; }
constexpr int b_off(int l) { return w_off(l) + w_size(l); }
constexpr int NPARAM = b_off(NLAYER - 1) + COUTP[NLAYER - 1];
constexpr int wt_size(int l) { return CINP[l] * kd(l); }
constexpr int wt_off(int l) { return l == 0 ? 0 : wt_off(l - 1) + wt_size(l - 1); }
constexpr int WT_TOTAL = wt_off(NLAYER - 1) + wt_size(NLAYER - 1);
constexpr int WCHUNK = 2048;                   // output pixels per weight-gradient partial sum
constexpr int ERR_INDEX = 1;

// per-sample element counts of the stored BF16 tensors
constexpr int act_elems(int l) { return HIN[l] * HIN[l] * CINP[l]; }      // input of layer l
constexpr int grad_elems(int l) { return HOUT[l] * HOUT[l] * COUTP[l]; }  // dL/dz_l

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
}
__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// FP32 parameters -> BF16 W (same offsets) and, per layer, the transposed
// BF16 weights WT_l[c][(3u+v) * Cout_p + o] = W_l[o][(3u+v) * Cin_p + c] used by
// the input gradient (zero for reduction indices >= 9 Cout_p).
template <int L>
__device__ __forceinline__ void prep_wt(const float* p, __bf16* wt, int r) {
    constexpr int cinp = CINP[L], coutp = COUTP[L], K = kp(L), KD = kd(L);
    const int c = r / KD, kk = r % KD;
    float w = 0.f;
    if (kk < 9 * coutp) w = p[w_off(L) + (kk % coutp) * K + (kk / coutp) * cinp + c];
    wt[wt_off(L) + r] = (__bf16)w;
}
__global__ void k_prep(const float* p, __bf16* wbf, __bf16* wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPARAM) wbf[i] = (__bf16)p[i];
    if (i >= WT_TOTAL) return;
    if (i < wt_off(1)) prep_wt<0>(p, wt, i);
    else if (i < wt_off(2)) prep_wt<1>(p, wt, i - wt_off(1));
    else if (i < wt_off(3)) prep_wt<2>(p, wt, i - wt_off(2));
    else if (i < wt_off(4)) prep_wt<3>(p, wt, i - wt_off(3));
    else prep_wt<4>(p, wt, i - wt_off(4));
}

// Gather the 9 patterns of each neighbourhood (nbr: B x 9 indices into the
// n_pat patterns of 64 x 64) and store log(1 + max(I, 0)) as BF16 NHWC with 16
// channels (9 used).  An index outside [0, n_pat) raises ERR_INDEX and reads
// as an all-zero pattern.
__global__ void k_input(const float* pat, int n_pat, const int* nbr, int B, __bf16* X0, int* err) {
    const int n = B * IN * IN;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int b = q / (IN * IN), yx = q % (IN * IN);
        bf16x8 lo, hi = zero8();
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int j = nbr[b * NB + c];
            float v = 0.f;
            if (j >= 0 && j < n_pat) v = log1pf(fmaxf(pat[(size_t)j * IN * IN + yx], 0.f));
            else if (yx == 0) atomicOr(err, ERR_INDEX);
            if (c < 8) lo[c] = (__bf16)v;
            else hi[0] = (__bf16)v;
        }
        bf16x8* dst = reinterpret_cast<bf16x8*>(X0 + (size_t)q * 16);
        dst[0] = lo;
        dst[1] = hi;
    }
}

// Forward convolution of layer L over B samples:
//   z[p][o] = bias[o] + sum_k W[o][k] Xcol[k][p],   Y = bf16(max(z, 0))  (L < 4)
//   out[p] = z[p][0]                                                   (L = 4)
// One wave per 16 output pixels and all output channels.
template <int L>
__global__ __launch_bounds__(256) void k_fwd(const __bf16* X, const __bf16* W, const float* bias, __bf16* Y,
                                             float* out, int B) {
    constexpr int cinp = CINP[L], coutp = COUTP[L], s = STRIDE[L], hin = HIN[L], hout = HOUT[L], K = kp(L);
    constexpr int MT = coutp / 16;
    const int lane = threadIdx.x % 64, g = lane / 16, n = lane % 16;
    const int p0 = (blockIdx.x * 4 + threadIdx.x / 64) * 16;
    if (p0 >= B * hout * hout) return;
    const int p = p0 + n;
    const int b = p / (hout * hout), yo = (p / hout) % hout, xo = p % hout;
    floatx4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int k0 = 0; k0 < K; k0 += 32) {
        const int k = k0 + 8 * g;
        bf16x8 bv = zero8();
        if (k < 9 * cinp) {
            const int tap = k / cinp, c0 = k % cinp;
            const int yi = yo * s + tap / 3 - 1, xi = xo * s + tap % 3 - 1;
            if (yi >= 0 && yi < hin && xi >= 0 && xi < hin) bv = ld8(X + (((size_t)b * hin + yi) * hin + xi) * cinp + c0);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(ld8(W + (mt * 16 + n) * K + k), bv, acc[mt]);
    }
    if constexpr (L < NLAYER - 1) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            bf16x4 y4;
#pragma unroll
            for (int r = 0; r < 4; ++r) y4[r] = (__bf16)fmaxf(acc[mt][r] + bias[mt * 16 + 4 * g + r], 0.f);
            *reinterpret_cast<bf16x4*>(Y + (size_t)p * coutp + mt * 16 + 4 * g) = y4;
        }
    } else {
        if (g == 0) out[p] = acc[0][0] + bias[0];
    }
}

// Mean squared error over n outputs, two deterministic passes in FP64.
__global__ __launch_bounds__(256) void k_mse_partial(const float* out, const float* target, int n, double* part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = (double)out[i] - (double)target[i];
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_mse_final(const double* part, int nblk, int n, double* loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    *loss = s / n;
}

// dL/dz_4 = bf16(2 (out - target) / n) in channel 0 of 16
__global__ void k_mse_grad(const float* out, const float* target, int n, __bf16* G4) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        bf16x8 lo = zero8();
        lo[0] = (__bf16)(2.0f * (out[i] - target[i]) / (float)n);
        bf16x8* dst = reinterpret_cast<bf16x8*>(G4 + (size_t)i * 16);
        dst[0] = lo;
        dst[1] = zero8();
    }
}

// Weight and bias gradient of layer L over one chunk of WCHUNK output pixels:
//   part[chunk][o * K + k] = sum_{p in chunk} G[p][o] Xcol[k][p]
//   part[chunk][Cout_p * K + o] = sum_{p in chunk} G[p][o]        (bias)
// A workgroup covers one chunk and WG_NT(L) consecutive 16-wide reduction
// tiles (blockIdx.y) for all output channels.  For every 32 pixels it stages
// G^T and the im2col rows Xcol of its reduction range in LDS, pixel-fastest
// (16-byte global loads of 8 channels, written out per channel), so each MFMA
// operand, 8 consecutive pixels of one row, is one 16-byte LDS read; the pixel
// sum is the MFMA reduction.  The waves holding the k = 0..15 tiles also add up
// their G operands for the bias, in a fixed order (own pixels, then lanes 16
// and 32 apart).
template <int L> constexpr int wg_nt() { return (kp(L) / 16 + 2) / 3; }

template <int L>
__global__ __launch_bounds__(256) void k_wgrad(const __bf16* G, const __bf16* X, float* part, int B) {
    constexpr int cinp = CINP[L], coutp = COUTP[L], s = STRIDE[L], hin = HIN[L], hout = HOUT[L], K = kp(L);
    constexpr int MT = coutp / 16, NT = K / 16, NTW = wg_nt<L>(), KW = 16 * NTW;
    constexpr int TPW = (MT * NTW + 3) / 4;            // tiles per wave
    constexpr int PITCH = 40;                          // bf16 per staged row: 32 pixels, 80 B (16-B aligned rows)
    __shared__ __align__(16) __bf16 gs[coutp * PITCH];
    __shared__ __align__(16) __bf16 xs[KW * PITCH];
    const int lane = threadIdx.x % 64, g = lane / 16, n = lane % 16, wave = threadIdx.x / 64;
    const int chunk = blockIdx.x, nt0 = blockIdx.y * NTW, ntw = min(NTW, NT - nt0), k0 = 16 * nt0;
    const int P = B * hout * hout;                     // the last chunk may be partial
    const int pbase = chunk * WCHUNK, qend = min(WCHUNK, P - pbase);
    floatx4 acc[TPW];
    float bs[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        bs[t] = 0.f;
    }
    // the pieces this thread stages, two pixels each (16 bytes = 8 channels
    // of each): G^T items it = tid + 256 j (16 pixel pairs x coutp / 8 channel
    // groups), Xcol items likewise (16 pixel pairs x KW / 8 row groups; 8
    // consecutive k share a tap, cinp being a multiple of 8).  A pair goes to
    // LDS as 8 dwords (channel e of both pixels); the next 32 pixels' pieces
    // are loaded while the MFMAs run.
    constexpr int NGI = 16 * (coutp / 8), NXI = 16 * (KW / 8);
    constexpr int NG = (NGI + 255) / 256, NX = (NXI + 255) / 256;
    bf16x8 gv[NG][2], xv[NX][2];
    auto xload = [&](int p, int k) -> bf16x8 {
        const int tap = k / cinp, c = k % cinp;
        const int b = p / (hout * hout), yo = (p / hout) % hout, xo = p % hout;
        const int yi = yo * s + tap / 3 - 1, xi = xo * s + tap % 3 - 1;
        if (p < P && yi >= 0 && yi < hin && xi >= 0 && xi < hin) return ld8(X + (((size_t)b * hin + yi) * hin + xi) * cinp + c);
        return zero8();
    };
    auto fetch = [&](int p0) {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int it = threadIdx.x + 256 * j, cg = it / 16, p = p0 + 2 * (it % 16);
#pragma unroll
            for (int h = 0; h < 2; ++h)
                gv[j][h] = it < NGI && p + h < P ? ld8(G + (size_t)(p + h) * coutp + 8 * cg) : zero8();
        }
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            const int it = threadIdx.x + 256 * j, kg = it / 16, p = p0 + 2 * (it % 16), k = k0 + 8 * kg;
            const bool use = it < NXI && kg < 2 * ntw && k < 9 * cinp;
#pragma unroll
            for (int h = 0; h < 2; ++h) xv[j][h] = use ? xload(p + h, k) : zero8();
        }
    };
    // channel e of a pixel pair (a: first pixel, low half) as one dword
    auto pair = [](const bf16x8& a, const bf16x8& b, int e) -> uint32_t {
        const u32x4 ua = __builtin_bit_cast(u32x4, a), ub = __builtin_bit_cast(u32x4, b);
        const uint32_t x = ua[e >> 1], y = ub[e >> 1];
        return (e & 1) ? (x >> 16) | (y & 0xffff0000u) : (x & 0xffffu) | (y << 16);
    };
    uint32_t* gs32 = reinterpret_cast<uint32_t*>(gs);
    uint32_t* xs32 = reinterpret_cast<uint32_t*>(xs);
    fetch(pbase);
    for (int q0 = 0; q0 < qend; q0 += 32) {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int it = threadIdx.x + 256 * j, cg = it / 16, pq = it % 16;
            if (it < NGI) {
#pragma unroll
                for (int e = 0; e < 8; ++e) gs32[(8 * cg + e) * (PITCH / 2) + pq] = pair(gv[j][0], gv[j][1], e);
            }
        }
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            const int it = threadIdx.x + 256 * j, kg = it / 16, pq = it % 16;
            if (it < NXI) {
#pragma unroll
                for (int e = 0; e < 8; ++e) xs32[(8 * kg + e) * (PITCH / 2) + pq] = pair(xv[j][0], xv[j][1], e);
            }
        }
        __syncthreads();
        if (q0 + 32 < qend) fetch(pbase + q0 + 32);
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int i = wave + 4 * t, mt = i / NTW, ntl = i % NTW;
            if (i < MT * NTW && ntl < ntw) {
                const bf16x8 av = *reinterpret_cast<const bf16x8*>(gs + (mt * 16 + n) * PITCH + 8 * g);
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(xs + (ntl * 16 + n) * PITCH + 8 * g);
                acc[t] = mfma(av, bv, acc[t]);
                if (nt0 == 0 && ntl == 0) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) bs[t] += (float)av[e];
                }
            }
        }
        __syncthreads();
    }
    float* dst = part + (size_t)chunk * (w_size(L) + coutp);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int i = wave + 4 * t, mt = i / NTW, ntl = i % NTW;
        if (i < MT * NTW && ntl < ntw) {
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[(mt * 16 + 4 * g + r) * K + (nt0 + ntl) * 16 + n] = acc[t][r];
            if (nt0 == 0 && ntl == 0) {
                float b = bs[t];
                b += __shfl_xor(b, 16, 64);
                b += __shfl_xor(b, 32, 64);
                if (g == 0) dst[w_size(L) + mt * 16 + n] = b;
            }
        }
    }
}

// grad[i] += sum over chunks, in chunk order, of part[chunk][i], i < n.
// A block covers 32 entries with 8 threads each; thread t sums the chunks
// t, t + 8, ... and the 8 partial sums are added in thread order.
__global__ __launch_bounds__(256) void k_wreduce(const float* part, int nchunk, int n, float* grad) {
    __shared__ float sh[8][33];
    const int e = threadIdx.x % 32, t = threadIdx.x / 32;
    const int i = blockIdx.x * 32 + e;
    float s = 0.f;
    if (i < n)
        for (int ch = t; ch < nchunk; ch += 8) s += part[(size_t)ch * n + i];
    sh[t][e] = s;
    __syncthreads();
    if (t == 0 && i < n) {
        float r = sh[0][e];
#pragma unroll
        for (int q = 1; q < 8; ++q) r += sh[q][e];
        grad[i] += r;
    }
}

// Input gradient of layer L (L >= 1) through the ReLU of layer L-1:
//   Gprev[q][c] = bf16([X[q][c] > 0] sum_{tap, o} WT[c][tap * Cout_p + o] G[p_out(q, tap)][o])
// where output pixel p_out = ((y + 1 - u) / s, (x + 1 - v) / s) when that is an
// integer inside the output.  One wave per 16 input pixels and all channels
// (stride 2: 16 pixels of one parity class, see below).
template <int L>
__global__ __launch_bounds__(256) void k_dgrad(const __bf16* G, const __bf16* WT, const __bf16* X, __bf16* Gprev,
                                               int B) {
    constexpr int cinp = CINP[L], coutp = COUTP[L], s = STRIDE[L], hin = HIN[L], hout = HOUT[L], KD = kd(L);
    constexpr int MT = cinp / 16;
    const int lane = threadIdx.x % 64, g = lane / 16, n = lane % 16;
    const int wv = blockIdx.x * 4 + threadIdx.x / 64;
    if (wv * 16 >= B * hin * hin) return;
    int b, yi, xi;
    floatx4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
    if constexpr (s == 2) {
        // A wave takes 16 input pixels of one row and one column parity
        // (every other pixel of half a row): only the taps (u, v) with
        // y + 1 - u and x + 1 - v even meet an output pixel, the same for all
        // 16 (u = 1 for even rows, u = 0, 2 for odd ones; v likewise), so the
        // reduction runs over those 1, 2 or 4 taps in increasing order (the
        // other taps' products are zero) instead of all 9.
        static_assert(coutp == 32, "one 32-wide reduction step per tap");
        const int rem = wv % (hin * 4), px = (rem / 2) % 2, half = rem % 2;
        b = wv / (hin * 4);
        yi = rem / 4;
        xi = 2 * (16 * half + n) + px;
        const int u0 = (yi % 2 == 0) ? 1 : 0, du = (yi % 2 == 0) ? 3 : 2;   // u = 1, or u = 0, 2
        const int v0 = px == 0 ? 1 : 0, dv = px == 0 ? 3 : 2;
        for (int u = u0; u < 3; u += du)
            for (int v = v0; v < 3; v += dv) {
                const int tap = 3 * u + v, kk = tap * coutp + 8 * g;
                const int ty = yi + 1 - u, tx = xi + 1 - v;
                bf16x8 bv = zero8();
                if (ty >= 0 && tx >= 0 && ty / 2 < hout && tx / 2 < hout)
                    bv = ld8(G + (((size_t)b * hout + ty / 2) * hout + tx / 2) * coutp + 8 * g);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(ld8(WT + (mt * 16 + n) * KD + kk), bv, acc[mt]);
            }
    } else {
        const int q = wv * 16 + n;
        b = q / (hin * hin);
        yi = (q / hin) % hin;
        xi = q % hin;
#pragma unroll 3
        for (int k0 = 0; k0 < KD; k0 += 32) {
            const int kk = k0 + 8 * g;
            bf16x8 bv = zero8();
            if (kk < 9 * coutp) {
                const int tap = kk / coutp, o0 = kk % coutp;
                const int ty = yi + 1 - tap / 3, tx = xi + 1 - tap % 3;
                if (ty >= 0 && tx >= 0 && ty % s == 0 && tx % s == 0 && ty / s < hout && tx / s < hout)
                    bv = ld8(G + (((size_t)b * hout + ty / s) * hout + tx / s) * coutp + o0);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(ld8(WT + (mt * 16 + n) * KD + kk), bv, acc[mt]);
        }
    }
    const int q = (b * hin + yi) * hin + xi;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const size_t o = (size_t)q * cinp + mt * 16 + 4 * g;
        const bf16x4 x4 = *reinterpret_cast<const bf16x4*>(X + o);
        bf16x4 g4;
#pragma unroll
        for (int r = 0; r < 4; ++r) g4[r] = (float)x4[r] > 0.f ? (__bf16)acc[mt][r] : (__bf16)0.0f;
        *reinterpret_cast<bf16x4*>(Gprev + o) = g4;
    }
}

// Adam on the FP32 parameter vector (PyTorch's form: bias-corrected moments,
// eps added to the corrected square root).
__global__ void k_adam(float* p, const float* gr, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2s) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = gr[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= (lr / bc1) * mi / (sqrtf(vi) / bc2s + eps);
    }
}

// Average the 32 x 32 patches (P of them, centred at round_half_even(centre),
// rows [cy - 16, cy + 16)) that cover each image pixel; uncovered pixels keep
// their value.  One thread per pixel, patches visited in order.
__global__ void k_stitch(const float* patches, const float* centres, int P, int H, int W, float* img) {
    const int n = H * W;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int y = i / W, x = i % W;
        float s = 0.f;
        int cnt = 0;
        for (int q = 0; q < P; ++q) {
            const int y0 = (int)rintf(centres[2 * q]) - OUT / 2, x0 = (int)rintf(centres[2 * q + 1]) - OUT / 2;
            if (y >= y0 && y < y0 + OUT && x >= x0 && x < x0 + OUT) {
                s += patches[(size_t)q * OUT * OUT + (y - y0) * OUT + (x - x0)];
                ++cnt;
            }
        }
        if (cnt) img[i] = s / (float)cnt;
    }
}

}  // namespace cnn
}  // namespace ptyr
