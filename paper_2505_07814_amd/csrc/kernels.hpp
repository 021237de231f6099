// kernels.hpp - gfx950 kernels of the multislice forward model, its loss, its
// gradient and the Adam step.  The fused per-(position, mode) kernels keep the
// whole N x N wave (N = 64 or 128) in registers across all slices and use LDS
// only for line exchanges and transposes (wave.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave.hpp"

namespace ptyr {

enum : int { ERR_BOUNDS = 1, ERR_NONFINITE = 2, ERR_ZERO_MEAN = 4, ERR_INDEX = 8 };

struct PosInfo {      // integer crop corner and sub-pixel shift of one batch row
    int ty, tx;       // ty < 0 marks a row that is skipped (patch out of bounds / bad index)
    float dry, drx;
    int row;          // validated row of pos / tilt / measured data (0 when skipped)
    int pad[3];
};

// Arguments shared by the fused forward / gradient kernels.
struct WaveArgs {
    const float2* Oc;      // S x H x W complex transmission a exp(i phase)
    const float2* Phat;    // M x N x N probe spectra F[P_m] (orthonormal)
    const PosInfo* pinfo;  // B, with validated rows
    const float* tilt;     // rows of (th_y, th_x)
    const float* dz;       // 1
    float2* store;         // B x M x nck x N x N kept waves (nullable)
    int ckK;               // keep phi_s for s % ckK == 0 (ckK > S: none kept)
    int nck;               // kept waves per chain
    int B, M, S, H, W;
    double dx, lam;
    int global_tilt;
    // forward output
    float* Imode;          // B x M x N x N, fftshifted
    // gradient inputs / outputs
    const float* wgt;      // B x N x N fftshifted, 2 dL/dI
    float2* gO;            // B x M x S x N x N object-patch gradients
    float2* gPhat;         // B x M x N x N probe-spectrum gradients
    float* part;           // B x M x 8 scalar partial sums
};

// ------------------------------------------------------------------ tables
// Per-workgroup LDS tables: twiddles and the separable propagator / shift.
template <int N> struct Tables {
    float4 tw[N];          // per-lane twiddles: tw[c*16 + b] = exp(-2 pi i c b / N)
    float4 hy[N], hx[N];   // propagator factors along y and x (unscaled)
    float dry, drx;        // sub-pixel shift of the position
};

// shift ramp factor exp(-2 pi i q_n dr) (used once per chain, computed in place)
template <int N> __device__ __forceinline__ float2 ramp(int n, float dr) {
    float s, c;
    sincospif(-2.0f * (float)sfreq<N>(n) / N * dr, &s, &c);
    return make_float2(c, s);
}

template <int N>
__device__ void build_tables(Tables<N>& t, const WaveArgs& a, const PosInfo& pi, float thy, float thx,
                             float dz) {
    constexpr int T = N * N / 16;
    const double pi_d = 3.14159265358979323846;
    if (threadIdx.x == 0) { t.dry = pi.dry; t.drx = pi.drx; }
    for (int i = threadIdx.x; i < 3 * N; i += T) {
        int which = i / N, n = i % N;
        double q = (double)sfreq<N>(n) / N;            // cycles per pixel
        double k = q / a.dx;                            // 1/angstrom
        double ph;
        if (which == 0) ph = -2.0 * pi_d * (double)((n / 16) * (n % 16)) / N;
        else if (which == 1) ph = -pi_d * a.lam * dz * k * k + 2.0 * pi_d * dz * k * tan((double)thy);
        else ph = -pi_d * a.lam * dz * k * k + 2.0 * pi_d * dz * k * tan((double)thx);
        double s, c;
        sincos(ph, &s, &c);
        float4 w = unit_pair(c, s);
        if (which == 0) t.tw[n] = w;
        else if (which == 1) t.hy[n] = w;
        else t.hx[n] = w;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ steps
// chi = O_s[t + (y, x)] * v  in layout (D, NAT)
template <int N, int D>
__device__ __forceinline__ void transmit(float2 (&v)[16], const float2* Os, int W, int ty, int tx, int l, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, D, NAT>(l, c, r, y, x);
        v[r] = cmul(v[r], Os[(size_t)(ty + y) * W + tx + x]);
    }
}

// F^-1_line [ h * F_line [v] ] along the lines of direction D, times scale
template <int N>
__device__ __forceinline__ void line_prop(float2 (&v)[16], float2* lds, const float4* tw, const float4* h,
                                          float scale, int l, int c) {
    nat2mid<N, -1>(v, lds, tw, l, c);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cscale(tmul<false>(v[r], h[line_pos<N, MID>(c, r)]), scale);
    mid2nat<N, +1>(v, lds, tw, l, c);
}

// One propagation between slices, separable: F^-1 H F = (F^-1 h_y F)_y (F^-1 h_x F)_x.
// The field enters in (st, NAT) and leaves in (other, NAT); returns the new state.
template <int N>
__device__ __forceinline__ int propagate(float2 (&v)[16], int st, float2* lds, const Tables<N>& t, int l, int c) {
    const float sc = 1.0f / N;
    if (st == COL) {
        line_prop<N>(v, lds, t.tw, t.hy, sc, l, c);
        relayout<N, COL, NAT, ROW, NAT>(v, lds, l, c);
        line_prop<N>(v, lds, t.tw, t.hx, sc, l, c);
        return ROW;
    } else {
        line_prop<N>(v, lds, t.tw, t.hx, sc, l, c);
        relayout<N, ROW, NAT, COL, NAT>(v, lds, l, c);
        line_prop<N>(v, lds, t.tw, t.hy, sc, l, c);
        return COL;
    }
}

template <int N>
__device__ __forceinline__ void transmit_state(float2 (&v)[16], int st, const float2* Os, int W, int ty, int tx,
                                               int l, int c) {
    if (st == COL) transmit<N, COL>(v, Os, W, ty, tx, l, c);
    else transmit<N, ROW>(v, Os, W, ty, tx, l, c);
}

// phi_0 = F^-1[ Phat_m * R ] (orthonormal), leaves in (COL, NAT)
template <int N>
__device__ __forceinline__ void shift_probe(float2 (&v)[16], const float2* Pm, float2* lds, const Tables<N>& t,
                                            int l, int c) {
    const float sc = 1.0f / N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int u = l, w = line_pos<N, MID>(c, r);
        v[r] = cscale(cmul(cmul(Pm[u * N + w], ramp<N>(u, t.dry)), ramp<N>(w, t.drx)), sc);
    }
    mid2nat<N, +1>(v, lds, t.tw, l, c);
    relayout<N, ROW, NAT, COL, MID>(v, lds, l, c);
    mid2nat<N, +1>(v, lds, t.tw, l, c);
}

// unnormalised 2-D DFT of sign -1 from (COL, NAT); leaves in (ROW, MID)
template <int N>
__device__ __forceinline__ void fft2_from_col(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    nat2mid<N, -1>(v, lds, tw, l, c);
    relayout<N, COL, MID, ROW, NAT>(v, lds, l, c);
    nat2mid<N, -1>(v, lds, tw, l, c);
}
// unnormalised 2-D DFT of sign -1 from (ROW, NAT); leaves in (COL, MID)
template <int N>
__device__ __forceinline__ void fft2_from_row(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    nat2mid<N, -1>(v, lds, tw, l, c);
    relayout<N, ROW, MID, COL, NAT>(v, lds, l, c);
    nat2mid<N, -1>(v, lds, tw, l, c);
}
// unnormalised 2-D inverse DFT from (ROW, MID); leaves in (COL, NAT)
template <int N>
__device__ __forceinline__ void ifft2_to_col(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    mid2nat<N, +1>(v, lds, tw, l, c);
    relayout<N, ROW, NAT, COL, MID>(v, lds, l, c);
    mid2nat<N, +1>(v, lds, tw, l, c);
}

template <int N>
__device__ __forceinline__ void store_wave_col(const float2 (&v)[16], float2* dst, int l, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, COL, NAT>(l, c, r, y, x);
        dst[y * N + x] = v[r];
    }
}
template <int N>
__device__ __forceinline__ void load_wave_col(float2 (&v)[16], const float2* src, int l, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, COL, NAT>(l, c, r, y, x);
        v[r] = src[y * N + x];
    }
}

// Incident wave of slice s in (COL, NAT): from the nearest kept wave (or the
// shifted probe when none is kept), re-running the slice steps in between
// with exactly the forward's code.
template <int N>
__device__ void incident_wave(float2 (&v)[16], int s, const WaveArgs& a, int j, int m, int ty, int tx, float2* lds,
                              const Tables<N>& t, int l, int c) {
    int s0;
    if (a.ckK <= a.S) {
        s0 = (s / a.ckK) * a.ckK;
        const float2* src = a.store + ((size_t)(j * a.M + m) * a.nck + s0 / a.ckK) * (N * N);
        load_wave_col<N>(v, src, l, c);
    } else {
        s0 = 0;
        shift_probe<N>(v, a.Phat + (size_t)m * N * N, lds, t, l, c);
    }
    int st = COL;
    for (int u = s0; u < s; ++u) {
        transmit_state<N>(v, st, a.Oc + (size_t)u * a.H * a.W, a.W, ty, tx, l, c);
        st = propagate<N>(v, st, lds, t, l, c);
    }
    if (st == ROW) relayout<N, ROW, NAT, COL, NAT>(v, lds, l, c);
}

// block-wide sum of NV floats, result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(float (&x)[NV], float* red) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x[k] += __shfl_xor(x[k], o, 64);
    const int w = threadIdx.x / 64, nw = blockDim.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[w * NV + k] = x[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) {
            float s = 0.f;
            for (int q = 0; q < nw; ++q) s += red[q * NV + k];
            x[k] = s;
        }
    __syncthreads();
}

// ------------------------------------------------------------------ kernels
// Forward: one workgroup per (batch row j, probe mode m).
template <int N>
__global__ __launch_bounds__(N * N / 16) void k_forward(WaveArgs a) {
    constexpr int L = N / 16;
    __shared__ float2 lds[WaveGeo<N>::LDS_SLOTS];
    __shared__ Tables<N> tab;
    const int l = threadIdx.x / L, c = threadIdx.x % L;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int j = wg / a.M, m = wg % a.M;
    const PosInfo pi = a.pinfo[j];
    float* Iout = a.Imode + (size_t)(j * a.M + m) * N * N;
    if (pi.ty < 0) {
        for (int i = threadIdx.x; i < N * N; i += blockDim.x) Iout[i] = 0.f;
        return;
    }
    const float* th = a.global_tilt ? a.tilt : a.tilt + 2 * pi.row;
    const float dz = *a.dz;
    build_tables<N>(tab, a, pi, th[0], th[1], dz);

    float2 v[16];
    shift_probe<N>(v, a.Phat + (size_t)m * N * N, lds, tab, l, c);
    int st = COL;
    for (int s = 0; s < a.S; ++s) {
        if (a.store && a.ckK <= a.S && s % a.ckK == 0) {
            float2* dst = a.store + ((size_t)(j * a.M + m) * a.nck + s / a.ckK) * (N * N);
            if (st == COL) store_wave_col<N>(v, dst, l, c);
            else {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    int y, x;
                    reg_yx<N, ROW, NAT>(l, c, r, y, x);
                    dst[y * N + x] = v[r];
                }
            }
        }
        transmit_state<N>(v, st, a.Oc + (size_t)s * a.H * a.W, a.W, pi.ty, pi.tx, l, c);
        if (s < a.S - 1) st = propagate<N>(v, st, lds, tab, l, c);
    }
    // far field |F chi|^2 / N^2, written with zero frequency at (N/2, N/2)
    const float s2 = 1.0f / ((float)N * N);
    if (st == COL) {
        fft2_from_col<N>(v, lds, tab.tw, l, c);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int y, x;
            reg_yx<N, ROW, MID>(l, c, r, y, x);
            Iout[((y + N / 2) % N) * N + (x + N / 2) % N] = cabs2(v[r]) * s2;
        }
    } else {
        fft2_from_row<N>(v, lds, tab.tw, l, c);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int y, x;
            reg_yx<N, COL, MID>(l, c, r, y, x);
            Iout[((y + N / 2) % N) * N + (x + N / 2) % N] = cabs2(v[r]) * s2;
        }
    }
}

// Gradient: one workgroup per (batch row j, probe mode m).  Walks the slices
// backwards (chain rule through Eq. 2-4), writing per-slice object-patch
// gradients, the probe-spectrum gradient and partial sums for the position,
// tilt and dz gradients.
template <int N>
__global__ __launch_bounds__(N * N / 16) void k_gradient(WaveArgs a) {
    constexpr int L = N / 16;
    __shared__ float2 lds[WaveGeo<N>::LDS_SLOTS];
    __shared__ Tables<N> tab;
    __shared__ float red[16 * 8];
    const int l = threadIdx.x / L, c = threadIdx.x % L;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int j = wg / a.M, m = wg % a.M;
    const PosInfo pi = a.pinfo[j];
    float* part = a.part + (size_t)(j * a.M + m) * 8;
    float2* gP = a.gPhat + (size_t)(j * a.M + m) * N * N;
    if (pi.ty < 0) {
        for (int i = threadIdx.x; i < N * N; i += blockDim.x) gP[i] = make_float2(0.f, 0.f);
        if (threadIdx.x < 8) part[threadIdx.x] = 0.f;
        return;   // the object-gradient scatter skips such rows
    }
    const float* th = a.global_tilt ? a.tilt : a.tilt + 2 * pi.row;
    const float dz = *a.dz;
    build_tables<N>(tab, a, pi, th[0], th[1], dz);
    const size_t HW = (size_t)a.H * a.W;
    const float inv_n = 1.0f / N, inv_n2 = 1.0f / ((float)N * N);

    float2 g[16], p[16];
    // G_chi_{S-1} = F^-1[ w * F[chi_{S-1}] ]   (w = 2 dL/dI)
    incident_wave<N>(g, a.S - 1, a, j, m, pi.ty, pi.tx, lds, tab, l, c);
    transmit<N, COL>(g, a.Oc + (size_t)(a.S - 1) * HW, a.W, pi.ty, pi.tx, l, c);
    fft2_from_col<N>(g, lds, tab.tw, l, c);
    const float* wj = a.wgt + (size_t)j * N * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, ROW, MID>(l, c, r, y, x);
        g[r] = cscale(g[r], wj[((y + N / 2) % N) * N + (x + N / 2) % N] * inv_n2);
    }
    ifft2_to_col<N>(g, lds, tab.tw, l, c);

    float acc_k2 = 0.f, acc_kx = 0.f, acc_ky = 0.f, acc_py = 0.f, acc_px = 0.f;
    const float dk = (float)(1.0 / (N * a.dx));
    for (int s = a.S - 1; s >= 0; --s) {
        const float2* Os = a.Oc + (size_t)s * HW;
        incident_wave<N>(p, s, a, j, m, pi.ty, pi.tx, lds, tab, l, c);
        float2* go = a.gO + ((size_t)(j * a.M + m) * a.S + s) * N * N;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int y, x;
            reg_yx<N, COL, NAT>(l, c, r, y, x);
            go[y * N + x] = cmulc(g[r], p[r]);                       // conj(phi) G_chi
            float2 o = Os[(size_t)(pi.ty + y) * a.W + pi.tx + x];
            g[r] = cmulc(g[r], o);                                    // G_phi = conj(O) G_chi
        }
        if (s > 0) {
            fft2_from_col<N>(p, lds, tab.tw, l, c);   // Y = F phi_s (raw)
            fft2_from_col<N>(g, lds, tab.tw, l, c);   // G^ = F G_phi (raw)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int y, x;
                reg_yx<N, ROW, MID>(l, c, r, y, x);
                float e = g[r].y * p[r].x - g[r].x * p[r].y;          // Im(G^ conj(Y))
                float ky = sfreq<N>(y) * dk, kx = sfreq<N>(x) * dk;
                acc_k2 = fmaf(e, kx * kx + ky * ky, acc_k2);
                acc_kx = fmaf(e, kx, acc_kx);
                acc_ky = fmaf(e, ky, acc_ky);
                g[r] = cscale(tmul<true>(tmul<true>(g[r], tab.hy[y]), tab.hx[x]), inv_n2);   // conj(H) G^ / N^2
            }
            ifft2_to_col<N>(g, lds, tab.tw, l, c);                    // G_chi_{s-1}
        } else {
            fft2_from_col<N>(g, lds, tab.tw, l, c);                   // G^_0 (raw)
            const float2* Pm = a.Phat + (size_t)m * N * N;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int y, x;
                reg_yx<N, ROW, MID>(l, c, r, y, x);
                float2 G0 = cscale(g[r], inv_n);
                float2 R = cmul(ramp<N>(y, tab.dry), ramp<N>(x, tab.drx));
                gP[y * N + x] = cmulc(G0, R);                          // conj(R) G^_0
                float2 z = cmulc(cmul(Pm[y * N + x], R), G0);          // Phat R conj(G^_0)
                acc_py = fmaf(z.y, (float)sfreq<N>(y) * inv_n, acc_py);
                acc_px = fmaf(z.y, (float)sfreq<N>(x) * inv_n, acc_px);
            }
        }
    }
    float sums[5] = {acc_k2 * inv_n2, acc_kx * inv_n2, acc_ky * inv_n2, acc_py, acc_px};
    block_sum<5>(sums, red);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 5; ++k) part[k] = sums[k];
        part[5] = part[6] = part[7] = 0.f;
    }
}

// Orthonormal 2-D DFT of sign SG of `count` N x N waves; out = or += result.
template <int N, int SG, bool ACC>
__global__ __launch_bounds__(N * N / 16) void k_fft2(const float2* in, float2* out) {
    constexpr int L = N / 16;
    __shared__ float2 lds[WaveGeo<N>::LDS_SLOTS];
    __shared__ float4 tw[N];
    const int l = threadIdx.x / L, c = threadIdx.x % L;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        double s, co;
        sincos(-2.0 * 3.14159265358979323846 * (double)((n / 16) * (n % 16)) / N, &s, &co);
        tw[n] = unit_pair(co, s);
    }
    __syncthreads();
    const float2* src = in + (size_t)blockIdx.x * N * N;
    float2* dst = out + (size_t)blockIdx.x * N * N;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, ROW, NAT>(l, c, r, y, x);
        v[r] = src[y * N + x];
    }
    nat2mid<N, SG>(v, lds, tw, l, c);
    relayout<N, ROW, MID, COL, NAT>(v, lds, l, c);
    nat2mid<N, SG>(v, lds, tw, l, c);
    const float sc = 1.0f / N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, COL, MID>(l, c, r, y, x);
        float2 val = cscale(v[r], sc);
        if (ACC) val = cadd(val, dst[y * N + x]);
        dst[y * N + x] = val;
    }
}

}  // namespace ptyr
