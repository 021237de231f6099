// ptyr.hip - libptyr: C ABI (include/ptyr.h), host validation and the
// element-wise / reduction kernels around the fused wave kernels.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ptyr.h"
#include "constrain.hpp"
#include "kernels.hpp"
#include "lines256.hpp"

using namespace ptyr;

namespace {

constexpr int NPART = 512;         // loss partial-sum blocks
constexpr double POISSON_EPS = 1e-6;

// ------------------------------------------------------------------ small kernels
__global__ void k_zero(float* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// O = a exp(i phase) (accurate sincos) for the n pixels, thread t0 of
// `stride` taking every stride-th one: four pixels at a time from 16-byte
// loads, two quads per thread issued before either is stored, where the
// parameters are 16-byte aligned (Oc is: the workspace is 256-byte aligned);
// pixel by pixel otherwise, and for the tail.
__device__ __forceinline__ void transmission(const float* __restrict__ amp, const float* __restrict__ phase,
                                             float2* __restrict__ Oc, size_t n, size_t t0, size_t stride) {
    size_t done = 0;
    if (((reinterpret_cast<uintptr_t>(amp) | reinterpret_cast<uintptr_t>(phase)) & 15) == 0) {
        const float4* a4 = reinterpret_cast<const float4*>(amp);
        const float4* p4 = reinterpret_cast<const float4*>(phase);
        float4* o4 = reinterpret_cast<float4*>(Oc);
        const size_t nq = n / 4;
        auto quad = [&](size_t q, const float4& a, const float4& ph) {
            float s0, c0, s1, c1, s2, c2, s3, c3;
            sincosf(ph.x, &s0, &c0);
            sincosf(ph.y, &s1, &c1);
            sincosf(ph.z, &s2, &c2);
            sincosf(ph.w, &s3, &c3);
            o4[2 * q] = make_float4(a.x * c0, a.x * s0, a.y * c1, a.y * s1);
            o4[2 * q + 1] = make_float4(a.z * c2, a.z * s2, a.w * c3, a.w * s3);
        };
        for (size_t q = t0; q < nq; q += 2 * stride) {
            const bool two = q + stride < nq;
            const float4 a = a4[q], ph = p4[q];
            const float4 a1 = two ? a4[q + stride] : a, ph1 = two ? p4[q + stride] : ph;
            quad(q, a, ph);
            if (two) quad(q + stride, a1, ph1);
        }
        done = nq * 4;
    }
    for (size_t i = done + t0; i < n; i += stride) {
        float s, c;
        sincosf(phase[i], &s, &c);
        const float a = amp[i];
        Oc[i] = make_float2(a * c, a * s);
    }
}

// O = a exp(i phase) for the whole object
__global__ void k_transmission(const float* amp, const float* phase, float2* Oc, size_t n) {
    transmission(amp, phase, Oc, n, blockIdx.x * (size_t)blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x);
}

// true when batch row j repeats the row of an earlier batch row (a gradient
// batch needs distinct rows: their position / tilt gradient updates would race)
__device__ bool repeated_row(int j, const int* idx) {
    const int row = idx[j];
    for (int i = 0; i < j; ++i)
        if (idx[i] == row) return true;
    return false;
}

// crop corner (round half to even) and sub-pixel shift of batch row j; with
// `distinct`, a row already used by an earlier batch row is skipped as a bad
// index
__device__ void position_info(int j, const float* pos, const int* idx, int n_rows, int N, int H, int W,
                              PosInfo* out, int* err, int distinct) {
    PosInfo pi;
    pi.ty = -1; pi.tx = -1; pi.dry = 0.f; pi.drx = 0.f; pi.row = 0;
    pi.pad[0] = pi.pad[1] = pi.pad[2] = 0;
    int row = idx ? idx[j] : j;
    if (row < 0 || row >= n_rows || (distinct && idx && repeated_row(j, idx))) {
        atomicOr(err, ERR_INDEX);
        out[j] = pi;
        return;
    }
    float py = pos[2 * row], px = pos[2 * row + 1];
    bool ok = isfinite(py) && isfinite(px);
    if (ok) {
        float ry = rintf(py), rx = rintf(px);
        float half = (float)(N / 2);
        ok = ry - half >= 0.f && rx - half >= 0.f && ry + half <= (float)H && rx + half <= (float)W;
        if (ok) {
            pi.ty = (int)ry - N / 2;
            pi.tx = (int)rx - N / 2;
            pi.dry = py - ry;
            pi.drx = px - rx;
            pi.row = row;
        }
    }
    if (!ok) atomicOr(err, ERR_BOUNDS);
    out[j] = pi;
}
__global__ void k_positions(const float* pos, const int* idx, int n_rows, int B, int N, int H, int W,
                            PosInfo* out, int* err, int distinct) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < B) position_info(j, pos, idx, n_rows, N, H, W, out, err, distinct);
}

// distinct rows for a gradient that reuses an earlier forward's positions:
// a repeated row is flagged (ptyr_sync reports PTYR_E_ARG) and skipped
__global__ void k_check_distinct(const int* idx, int B, PosInfo* pinfo, int* err) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < B; j += gridDim.x * blockDim.x)
        if (repeated_row(j, idx)) {
            atomicOr(err, ERR_INDEX);
            pinfo[j].ty = -1;
        }
}

// The work a batch shares, in one launch (N = 64, 128): workgroups 0 .. M-1
// transform the probe modes (long, one compute unit each), the others form
// the transmission of every slice, and the first of them the positions, so
// the transform overlaps the streaming pass instead of following it.
template <int N>
__global__ __launch_bounds__(N * N / 16) void k_prepare(const float* amp, const float* phase, float2* Oc, size_t nobj, const float* pos, const int* idx, int n_rows,
                                                        int B, int H, int W, PosInfo* pinfo, int* err,
                                                        const float2* probe, float2* Phat, int M, int distinct) {
    const int b = blockIdx.x;
    if (b < M) {
        fft2_block<N, -1, false>(probe + (size_t)b * N * N, Phat + (size_t)b * N * N);
        return;
    }
    const int nb = gridDim.x - M;
    if (b == M)
        for (int j = threadIdx.x; j < B; j += blockDim.x)
            position_info(j, pos, idx, n_rows, N, H, W, pinfo, err, distinct);
    transmission(amp, phase, Oc, nobj, (size_t)(b - M) * blockDim.x + threadIdx.x, (size_t)nb * blockDim.x);
}

// fftshift index of an N x N array (its own inverse for even N)
__device__ __forceinline__ int shift_index(int q, int N) {
    int y = q / N, x = q % N;
    return ((y + N / 2) % N) * N + (x + N / 2) % N;
}

// I[j] (zero frequency at (N/2, N/2)) = sum_m Imode[j][m] (zero frequency at (0, 0)), fixed order
__global__ void k_modesum(const float* Imode, float* I, int B, int M, int N) {
    const int NN = N * N;
    size_t n = (size_t)B * NN;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        size_t j = e / NN;
        int q = (int)(e % NN);
        const float* src = Imode + j * M * NN + shift_index(q, N);
        float s = 0.f;
        for (int m = 0; m < M; ++m) s += src[(size_t)m * NN];
        I[e] = s;
    }
}

__device__ __forceinline__ double powp(double v, double p) {
    if (p == 1.0) return v;
    if (p == 0.5) return sqrt(v);
    return pow(v, p);
}
// v^(p-1) for v > 0
__device__ __forceinline__ double powm1(double v, double p) {
    if (p == 1.0) return 1.0;
    if (p == 0.5) return 1.0 / sqrt(v);
    return pow(v, p - 1.0);
}

// The data terms of the loss (Eq. 5 / Eq. 6, or their weighted sum of
// Eq. 9): term t has kind k[t], power p[t] and weight w[t]; n = 1 or 2.
struct LossTerms {
    int n;
    int k[2];
    double p[2], w[2];
};

// per-pixel pieces of data term (kind, p) at model value I and measured value
// Em (both clamped at 0): the summand of the term's mean, dL/dA without the
// batch factor, and dL/dI without it
struct TermVal {
    double E, R, dI;
};
__device__ __forceinline__ TermVal term_val(int kind, double p, double Iv, double Em) {
    const double A = powp(Iv, p), E = powp(Em, p);
    TermVal t;
    t.E = E;
    double dA;
    if (kind == PTYR_LOSS_GAUSSIAN) {
        t.R = (A - E) * (A - E);
        dA = A - E;
    } else {
        t.R = E * log(A + POISSON_EPS) - A;
        dA = -(E / (A + POISSON_EPS) - 1.0);
    }
    t.dI = p == 1.0 ? dA : (Iv > 0.0 ? dA * p * powm1(Iv, p) : 0.0);
    return t;
}

// deterministic block sum of NP doubles per thread into part[NP * block + k]
template <int NP>
__device__ __forceinline__ void block_partials(double (&v)[NP], double* part) {
    __shared__ double sh[NP * 256];
    for (int k = 0; k < NP; ++k) sh[k * 256 + threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < NP; ++k) sh[k * 256 + threadIdx.x] += sh[k * 256 + threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < NP; ++k) part[NP * blockIdx.x + k] = sh[k * 256];
}

// loss partial sums per block: E_0, R_0, E_1, R_1 (term means' summands) and
// the count of non-finite inputs
constexpr int NLP = 5;

// pass 1 of the loss: per-block partial sums (ptyr_loss; inside the step
// k_loss_rows does this per row range)
__global__ __launch_bounds__(256) void k_loss_partial(const float* Im, const float* Ie, const int* midx, int n_meas,
                                                      int B, int NN, LossTerms lt, double* part, int* err) {
    double v[NLP] = {0, 0, 0, 0, 0};
    size_t n = (size_t)B * NN;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        size_t j = e / NN, q = e % NN;
        long row = midx ? (long)midx[j] : (long)j;
        if (row < 0 || row >= n_meas) {
            if (q == 0) atomicOr(err, ERR_INDEX);
            continue;
        }
        double I = Im[e], Em = Ie[(size_t)row * NN + q];
        if (!isfinite(I) || !isfinite(Em)) { v[4] += 1.0; continue; }
        I = fmax(I, 0.0); Em = fmax(Em, 0.0);
        for (int t = 0; t < lt.n; ++t) {
            const TermVal tv = term_val(lt.k[t], lt.p[t], I, Em);
            v[2 * t] += tv.E;
            v[2 * t + 1] += tv.R;
        }
    }
    block_partials<NLP>(v, part);
}

// pass 2: fixed-order totals, loss and the gradient scales.  Per term t
//   Gaussian: L_t = sqrt(D)/Z, dL/dA = (A-E) / (K sqrt(D) Z)
//   Poisson : L_t = -mean(E log(A+eps) - A)/Z, dL/dA = -(E/(A+eps) - 1)/(K Z)
// and L = sum_t w_t L_t.  scal[5 + t] = w_t c_t (the batch factor of term t,
// which the per-pixel dI of term_val is missing); scal[1] = the factor the
// gradient reductions apply to the weights of k_loss_rows (w_0 c_0, or 1
// when two terms are folded into the weights by k_loss_mix); scal[2] = Z_0.
__global__ void k_loss_final(const double* part, int nblk, double K, LossTerms lt, int check, double* scal,
                             double* loss_out, int* err, const double* spart, int nsp, double spw) {
    __shared__ double sh[NLP * 256];
    double s[NLP] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int k = 0; k < NLP; ++k) s[k] += part[NLP * b + k];
    for (int k = 0; k < NLP; ++k) sh[k * 256 + threadIdx.x] = s[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < NLP; ++k) sh[k * 256 + threadIdx.x] += sh[k * 256 + threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double bad = sh[4 * 256];
        double L = 0.0, c[2] = {0.0, 0.0}, Z0 = 0.0;
        bool zero_mean = false;
        for (int t = 0; t < lt.n; ++t) {
            const double sE = sh[(2 * t) * 256], sR = sh[(2 * t + 1) * 256];
            const double Z = sE / K;
            if (t == 0) Z0 = Z;
            if (!(Z > 0.0)) { zero_mean = true; continue; }
            if (lt.k[t] == PTYR_LOSS_GAUSSIAN) {
                const double D = sR / K;
                L += lt.w[t] * sqrt(D) / Z;
                c[t] = D > 0.0 ? lt.w[t] / (K * sqrt(D) * Z) : 0.0;
            } else {
                L += lt.w[t] * (-(sR / K) / Z);
                c[t] = lt.w[t] / (K * Z);
            }
        }
        if (zero_mean) {
            atomicOr(err, ERR_ZERO_MEAN);
            L = 0.0; c[0] = c[1] = 0.0;
        }
        if (nsp > 0) {                                  // + sparsity term, sums in order
            double t = 0.0;
            for (int i = 0; i < nsp; ++i) t += spart[i];
            L += spw * t;
        }
        if (check && (bad > 0.0 || !isfinite(L))) atomicOr(err, ERR_NONFINITE);
        scal[0] = L;
        scal[1] = lt.n > 1 ? 1.0 : c[0];
        scal[2] = Z0;
        scal[5] = c[0];
        scal[6] = c[1];
        if (loss_out) *loss_out = L;
    }
}

// dL/dI per value, in the layout of I_model (ptyr_loss)
__global__ void k_loss_grad(const float* Im, const float* Ie, const int* midx, int n_meas, int B, int N,
                            LossTerms lt, const double* scal, float* dLdI) {
    const int NN = N * N;
    const double c0 = scal[5], c1 = scal[6];
    size_t n = (size_t)B * NN;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        size_t j = e / NN, q = e % NN;
        long row = midx ? (long)midx[j] : (long)j;
        if (row < 0 || row >= n_meas) {
            dLdI[e] = 0.f;
            continue;
        }
        const double I = fmax((double)Im[e], 0.0), Em = fmax((double)Ie[(size_t)row * NN + q], 0.0);
        double dI = c0 * term_val(lt.k[0], lt.p[0], I, Em).dI;
        if (lt.n > 1) dI += c1 * term_val(lt.k[1], lt.p[1], I, Em).dI;
        dLdI[e] = (float)dI;
    }
}

// Rows [row0, row0 + nr) of a batch once their forward chains are done, in
// one pass: the mode sum I (fftshifted, as k_modesum), per-block loss
// partial sums (as k_loss_partial) and the gradient weights w = 2 dL/dI of
// the first data term without its batch factor.  Imode, I, midx and w2 start
// at row row0's entries.  A fixed grid and a fixed element-to-block map keep
// the sums deterministic.
__global__ __launch_bounds__(256) void k_loss_rows(const float* Imode, float* I, const float* Ie, const int* midx,
                                                   int n_meas, int nr, int M, int N, LossTerms lt, int row0,
                                                   double* part, float* w2, int* err) {
    const int NN = N * N;
    double v[NLP] = {0, 0, 0, 0, 0};
    const size_t n = (size_t)nr * NN;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t j = e / NN;
        const int q = (int)(e % NN), qs = shift_index(q, N);
        const float* src = Imode + j * M * NN + qs;
        float sum = 0.f;
        for (int m = 0; m < M; ++m) sum += src[(size_t)m * NN];
        I[e] = sum;
        const long row = midx ? (long)midx[j] : (long)(row0 + j);
        float* w = w2 + j * NN + qs;
        if (row < 0 || row >= n_meas) {
            if (q == 0) atomicOr(err, ERR_INDEX);
            *w = 0.f;
            continue;
        }
        const float em = Ie[(size_t)row * NN + q];
        const double Iv = fmax((double)sum, 0.0), Em = fmax((double)em, 0.0);
        const TermVal t0 = term_val(lt.k[0], lt.p[0], Iv, Em);
        if (!isfinite(sum) || !isfinite(em)) v[4] += 1.0;
        else {
            v[0] += t0.E;
            v[1] += t0.R;
            if (lt.n > 1) {
                const TermVal t1 = term_val(lt.k[1], lt.p[1], Iv, Em);
                v[2] += t1.E;
                v[3] += t1.R;
            }
        }
        *w = (float)(2.0 * t0.dI);
    }
    block_partials<NLP>(v, part);
}

// Two data terms (Eq. 9): once both batch factors are known, the weights of
// rows [row0, row0 + B) become w = c_0 w + 2 c_1 dI_1 (scal[5], scal[6]; the
// reductions then apply scal[1] = 1).  I is the fftshifted mode sum.
__global__ void k_loss_mix(float* w2, const float* I, const float* Ie, const int* midx, int n_meas, int row0, int B,
                           int N, LossTerms lt, const double* scal) {
    const int NN = N * N;
    const double c0 = scal[5], c1 = scal[6];
    const size_t n = (size_t)B * NN;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t j = e / NN;
        const int q = (int)(e % NN);
        float* w = w2 + j * NN + shift_index(q, N);
        const long row = midx ? (long)midx[j] : (long)(row0 + j);
        if (row < 0 || row >= n_meas) continue;      // already 0 and reported
        const double Iv = fmax((double)I[e], 0.0), Em = fmax((double)Ie[(size_t)row * NN + q], 0.0);
        *w = (float)(c0 * (double)*w + 2.0 * c1 * term_val(lt.k[1], lt.p[1], Iv, Em).dI);
    }
}

// One Adam update of a parameter element (Kingma & Ba, Alg. 1 with the bias
// corrections folded into the step: bc1 = 1 - b1^t, bc2s = sqrt(1 - b2^t)).
__device__ __forceinline__ void adam_elem(float& p, float& m, float& v, float g, float lr, float b1, float b2,
                                          float eps, float bc1, float bc2s) {
    const float mi = b1 * m + (1.f - b1) * g;
    const float vi = b2 * v + (1.f - b2) * g * g;
    m = mi;
    v = vi;
    p -= (lr / bc1) * mi / (sqrtf(vi) / bc2s + eps);
}

// Adam of the object, fused into the last scatter of a step: the parameter
// whose gradient buffer is non-null is updated and its buffer cleared.
struct ObjAdam {
    float *amp, *phase;                     // the parameters (read, then updated in place)
    float *m_amp, *v_amp, *m_phase, *v_phase;
    float lr_amp, lr_phase, b1, b2, eps, bc1, bc2s;
    int gin;    // fused launch: 1 = rows [0, j0) were scattered first by an
                // assigning launch, whose sums are read on the tiles those rows
                // touch (nothing else of g_amp / g_phase is read or written)
    int assign; // unfused launch: 1 = write the sums to the tiles the rows touch
                // (the first scatter of a fused step), 0 = add them
};

// Offset of patch pixel (py, px) in a stored patch gradient.  N = 256 (line
// passes): row-major.  N = 64, 128: the fused gradient's register-major
// order, register r of thread t at r T + t (T = N^2 / 16 threads).  There
// thread t = 64 w + k + P c (line_of: wave w, P = 64 / L lines per wave,
// L = N / 16 lanes per line) holds column x = P w + k, rows y = c + L r, so
// pixel (y, x) sits at (y / L) T + 64 (x / P) + x mod P + P (y mod L).
__device__ __forceinline__ size_t patch_offset(int py, int px, int N) {
    if (N == 256) return (size_t)py * N + px;
    const int lgL = N == 128 ? 3 : 2, lgP = 6 - lgL, T = N * N / 16;
    return (size_t)(py >> lgL) * T + ((px >> lgP) << 6) + (px & ((1 << lgP) - 1)) + ((py & ((1 << lgL) - 1)) << lgP);
}

// Object gradient: each workgroup owns a 32 x 32 tile of one slice and sums,
// in batch order, the patch gradients of every (position, mode) of batch rows
// [j0, j1) covering it;
// then applies the chain rule to amplitude and phase (O = a exp(i phase)):
//   g_a += Re(conj(G) exp(i phase)),  g_phase += Im(G conj(O)).
// A thread owns one column of the tile and four rows 8 apart, so each load
// instruction reads two whole 256-byte tile rows of a patch; the loads of MB
// consecutive (position, mode) items are issued together before they are
// added (in item order), to keep enough bytes in flight per workgroup.  FUSE: the
// launch also takes every pixel's complete gradient (this sum, plus the
// buffer's on the tiles an earlier assigning scatter of rows [0, j0) wrote)
// through Adam (ObjAdam), untouched tiles included; the buffers are never
// cleared, as each step's first scatter writes before the fused one reads.
// MB: 8 when the probe modes come in eights, else 4 (fewer registers, more
// resident workgroups).
template <bool FUSE, int SCATTER_MB>
__global__ __launch_bounds__(256) void k_scatter_object(const float2* gO, const PosInfo* pinfo, int j0, int j1, int M,
                                                        int Mc, int S, int N, int H, int W, const float* amp,
                                                        const float* phase, const double* scale, float* g_amp,
                                                        float* g_phase, ObjAdam ad, float sp) {
    const int ntx = (W + 31) / 32;
    // blockIdx.y = o S + s: object mode o, slice s; patch-gradient entries o M .. o M + M - 1 of a
    // position (Mc per position: one per chain, or one per group of probe modes at N = 256)
    const int tile = blockIdx.x, s = blockIdx.y % S, om = (blockIdx.y / S) * M;
    const int y0 = (tile / ntx) * 32, x0 = (tile % ntx) * 32;
    const int x = x0 + (int)threadIdx.x % 32, yb = y0 + (int)threadIdx.x / 32;
    float2 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = make_float2(0.f, 0.f);
    bool touched = false;
    int cnt[4] = {0, 0, 0, 0};                 // patches covering the pixel (sparsity term)
    const size_t NN = (size_t)N * N;
    // Work items are the (row, mode) pairs of the rows whose patch covers the
    // tile, in row then mode order; SCATTER_MB consecutive items are loaded
    // together, so with few modes the loads of several rows are in flight.
    // The cursor (jc, mc) is the same for the whole workgroup; jc == j1 once
    // no item is left.
    int jc = j0 - 1, mc = M - 1;
    PosInfo pc = {0, 0, 0.f, 0.f, 0, {0, 0, 0}};
    auto advance = [&]() {
        if (++mc < M) return;
        mc = 0;
        for (++jc; jc < j1; ++jc) {
            pc = pinfo[jc];
            if (pc.ty < 0) continue;
            if (pc.ty >= y0 + 32 || pc.ty + N <= y0 || pc.tx >= x0 + 32 || pc.tx + N <= x0) continue;
            touched = true;
            if (sp != 0.f) {
                const int px = x - pc.tx;
                const bool xin = px >= 0 && px < N;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int py = yb + 8 * i - pc.ty;
                    cnt[i] += (xin && py >= 0 && py < N) ? 1 : 0;
                }
            }
            return;
        }
    };
    advance();
    // FUSE with gin: whether the assigning scatter of rows [0, j0) wrote this tile
    bool pre = false;
    if (FUSE && ad.gin)
        for (int j = 0; j < j0 && !pre; ++j) {
            const int ty = pinfo[j].ty, tx = pinfo[j].tx;
            pre = ty >= 0 && ty < y0 + 32 && ty + N > y0 && tx < x0 + 32 && tx + N > x0;
        }
    while (jc < j1) {
        float2 buf[SCATTER_MB][4];
#pragma unroll
        for (int mm = 0; mm < SCATTER_MB; ++mm) {
            const bool live = jc < j1;
            const int px = x - pc.tx;
            const bool xin = live && px >= 0 && px < N;
            const float2* src = gO + ((size_t)(jc * Mc + om + mc) * S + s) * NN;   // read only when xin
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int py = yb + 8 * i - pc.ty;
                const bool in = xin && py >= 0 && py < N;
                buf[mm][i] = in ? src[patch_offset(py, px, N)] : make_float2(0.f, 0.f);
            }
            if (live) advance();
        }
#pragma unroll
        for (int mm = 0; mm < SCATTER_MB; ++mm)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = cadd(acc[i], buf[mm][i]);
    }
    if ((!FUSE && !touched) || x >= W) return;
    const float sc = (float)*scale;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = yb + 8 * i;
        if (y >= H) continue;
        size_t o = ((size_t)blockIdx.y * H + y) * W + x;
        float ga = 0.f, gp = 0.f;
        if (!FUSE || touched) {
            const float ph = phase[o];
            float sn, cs;
            sincosf(ph, &sn, &cs);
            float a = amp[o];
            float2 G = cscale(acc[i], sc);
            ga = G.x * cs + G.y * sn;              // Re(conj(G) e^{i phi})
            gp = a * (G.y * cs - G.x * sn);        // Im(G conj(a e^{i phi}))
            if (sp != 0.f) gp += sp * (float)cnt[i] * (ph > 0.f ? 1.f : (ph < 0.f ? -1.f : 0.f));
        }
        if constexpr (!FUSE) {
            if (g_amp) g_amp[o] = ad.assign ? ga : g_amp[o] + ga;
            if (g_phase) g_phase[o] = ad.assign ? gp : g_phase[o] + gp;
        } else {
            if (g_amp) {
                const float gi = pre ? ga + g_amp[o] : ga;
                adam_elem(ad.amp[o], ad.m_amp[o], ad.v_amp[o], gi, ad.lr_amp, ad.b1, ad.b2, ad.eps, ad.bc1, ad.bc2s);
            }
            if (g_phase) {
                const float gi = pre ? gp + g_phase[o] : gp;
                adam_elem(ad.phase[o], ad.m_phase[o], ad.v_phase[o], gi, ad.lr_phase, ad.b1, ad.b2, ad.eps, ad.bc1,
                          ad.bc2s);
            }
        }
    }
}

constexpr int PAC_BLOCKS = 64;

// PACBED term, pass 1: per detector pixel q (zero frequency at (N/2, N/2)) the
// batch means of the model and measured patterns, R = Abar^p - Ebar^p, kept
// as pac[2q] = R, pac[2q + 1] = Abar; per-block partial sums of R^2.
__global__ __launch_bounds__(256) void k_pacbed_partial(const float* I, const float* Ie, const int* midx, int n_meas,
                                                        int row0, int B, int NN, double p, double* pac,
                                                        double* part) {
    double r2 = 0.0;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < NN; q += gridDim.x * blockDim.x) {
        double a = 0.0, e = 0.0;
        for (int j = 0; j < B; ++j) {
            a += (double)I[(size_t)j * NN + q];
            const long row = midx ? (long)midx[j] : (long)(row0 + j);
            if (row >= 0 && row < n_meas) e += (double)Ie[(size_t)row * NN + q];
        }
        a = fmax(a / B, 0.0);
        e = fmax(e / B, 0.0);
        const double R = powp(a, p) - powp(e, p);
        pac[2 * q] = R;
        pac[2 * q + 1] = a;
        r2 += R * R;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = r2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// PACBED pass 2: L_pac = sqrt(<R^2>_D) / Z added (times w) to the loss;
// scal[3] = the gradient factor w p / (NN sqrt(D) Z B).  fold: the batch
// factor of the data term (scal[1]) moves to scal[4] and scal[1] becomes 1,
// for weights that carry both terms.
__global__ void k_pacbed_final(const double* part, int nblk, int NN, int B, double p, double w, double* scal,
                               double* loss_out, int fold) {
    if (threadIdx.x != 0) return;
    double D = 0.0;
    for (int b = 0; b < nblk; ++b) D += part[b];
    D /= NN;
    const double Z = scal[2];
    const double L = Z > 0.0 ? sqrt(D) / Z : 0.0;
    scal[0] += w * L;
    if (loss_out) *loss_out += w * L;
    scal[3] = (D > 0.0 && Z > 0.0) ? w * p / ((double)NN * sqrt(D) * Z * B) : 0.0;
    if (fold) {
        scal[4] = scal[1];
        scal[1] = 1.0;
    }
}

// PACBED pass 3: out = mul * out + fac * scal[3] R Abar^(p-1) for every row,
// mul = scal[4] (fold) or 1; the adjoint's weights (fac 2, unshifted layout)
// or ptyr_loss's dL/dI (fac 1, shifted layout).
__global__ void k_pacbed_grad(float* out, int B, int N, double p, const double* pac, const double* scal, int fold,
                              float fac, int unshift) {
    const int NN = N * N;
    const size_t n = (size_t)B * NN;
    const double mul = fold ? scal[4] : 1.0, sp = scal[3];
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t j = e / NN;
        const int q = (int)(e % NN);
        const double R = pac[2 * q], a = pac[2 * q + 1];
        const double d = p == 1.0 ? R : (a > 0.0 ? R * powm1(a, p) : 0.0);
        float* o = out + j * NN + (unshift ? shift_index(q, N) : q);
        *o = (float)(mul * (double)*o + (double)fac * sp * d);
    }
}

// Sparsity term: the sum of |phase| over the object patch of batch row j in
// slice s (one workgroup per (j, s), double), for the loss.
__global__ __launch_bounds__(256) void k_sparse_partial(const float* phase, const PosInfo* pinfo, int S, int N, int H,
                                                        int W, double* part) {
    const int j = blockIdx.x, s = blockIdx.y;
    const PosInfo pi = pinfo[j];
    double acc = 0.0;
    if (pi.ty >= 0)
        for (int e = threadIdx.x; e < N * N; e += blockDim.x)
            acc += fabs((double)phase[((size_t)s * H + pi.ty + e / N) * W + pi.tx + e % N]);
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)j * S + s] = sh[0];
}

// sum over batch rows of the probe-spectrum gradients (fixed order), times
// the batch factor
__global__ void k_sum_rows(const float2* src, float2* dst, int B, int M, int NN, const double* scale) {
    size_t n = (size_t)M * NN;
    const float sc = (float)*scale;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        float2 s = make_float2(0.f, 0.f);
        int j = 0;
        for (; j + 8 <= B; j += 8) {         // eight loads in flight, added in row order
            float2 t[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) t[q] = src[(size_t)(j + q) * n + e];
#pragma unroll
            for (int q = 0; q < 8; ++q) s = cadd(s, t[q]);
        }
        for (; j < B; ++j) s = cadd(s, src[(size_t)j * n + e]);
        dst[e] = cscale(s, sc);
    }
}

// position, tilt and dz gradients from the per-(row, mode) partial sums
//   g_rho   = 2 pi sum_m sum_k q Im(Phat R conj(G^_0))
//   g_th    = 2 pi dz sec^2(th) sum_s,m,k k Im(G^ conj(Y))
//   g_dz    = sum [-pi lam |k|^2 + 2 pi (k_x tan th_x + k_y tan th_y)] Im(G^ conj(Y))
// One thread per batch row (rows of a batch are distinct, so the row
// updates do not collide); dz and a global tilt are summed over rows in
// fixed order by a block tree.
__global__ __launch_bounds__(256) void k_param_grads(const double* part, int nblk, const PosInfo* pinfo, int B,
                                                     int M, const float* tilt, int global_tilt, const float* dzp,
                                                     double lam, const double* scale, float* g_pos, float* g_tilt,
                                                     float* g_dz) {
    __shared__ double sh[3][256];
    const double two_pi = 6.283185307179586;
    const double sc = *scale;                 // batch factor of the loss gradient
    const double dz = *dzp;
    double sdz = 0.0, sty = 0.0, stx = 0.0;
    for (int j = threadIdx.x; j < B; j += blockDim.x) {
        if (pinfo[j].ty < 0) continue;
        const int row = pinfo[j].row;
        double k2 = 0, kx = 0, ky = 0, py = 0, px = 0;
        for (int m = 0; m < M; ++m)
            for (int b = 0; b < nblk; ++b) {
                const double* q = part + ((size_t)(j * M + m) * nblk + b) * 8;
                k2 += q[0]; kx += q[1]; ky += q[2]; py += q[3]; px += q[4];
            }
        const float* th = global_tilt ? tilt : tilt + 2 * row;
        const double ty = tan((double)th[0]), tx = tan((double)th[1]);
        const double cy = cos((double)th[0]), cx = cos((double)th[1]);
        k2 *= sc; kx *= sc; ky *= sc; py *= sc; px *= sc;
        sdz += -3.141592653589793 * lam * k2 + two_pi * (tx * kx + ty * ky);
        const double gy = two_pi * dz * ky / (cy * cy), gx = two_pi * dz * kx / (cx * cx);
        if (global_tilt) { sty += gy; stx += gx; }
        else if (g_tilt) { g_tilt[2 * row] += (float)gy; g_tilt[2 * row + 1] += (float)gx; }
        if (g_pos) { g_pos[2 * row] += (float)(two_pi * py); g_pos[2 * row + 1] += (float)(two_pi * px); }
    }
    sh[0][threadIdx.x] = sdz; sh[1][threadIdx.x] = sty; sh[2][threadIdx.x] = stx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (global_tilt && g_tilt) { g_tilt[0] += (float)sh[1][0]; g_tilt[1] += (float)sh[2][0]; }
        if (g_dz) g_dz[0] += (float)sh[0][0];
    }
}

// Adam (PyTorch's form): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= (lr / bc1) * m / (sqrt(v) / sqrt(bc2) + eps)
// All parameter blocks of a step in one launch: segment k covers elements
// [off[k], off[k+1]) of the concatenated index range.  Each gradient entry
// is cleared once read, so the step's gradient buffers start the next step
// at zero; a segment with upd = 0 (learning rate 0) is only cleared.
constexpr int ADAM_SEGS = 6;
struct AdamSegs {
    float* p[ADAM_SEGS];
    float* g[ADAM_SEGS];
    float* m[ADAM_SEGS];
    float* v[ADAM_SEGS];
    size_t off[ADAM_SEGS + 1];
    float lr[ADAM_SEGS];
    int upd[ADAM_SEGS];
};
// the Adam constants of one step beside the segments
struct SegAdam {
    AdamSegs A;
    float b1, b2, eps, bc1, bc2s;
};
__global__ void k_adam_segs(AdamSegs a, float b1, float b2, float eps, float bc1, float bc2s) {
    const size_t n = a.off[ADAM_SEGS];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        int k = 0;
#pragma unroll
        for (int q = 1; q < ADAM_SEGS; ++q)
            if (i >= a.off[q]) k = q;
        const size_t e = i - a.off[k];
        const float gi = a.g[k][e];
        a.g[k][e] = 0.f;
        if (!a.upd[k]) continue;
        adam_elem(a.p[k][e], a.m[k][e], a.v[k][e], gi, a.lr[k], b1, b2, eps, bc1, bc2s);
    }
}

// ------------------------------------------------------------------ host helpers
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// object modes (0 in the geometry means one) and chain modes per batch row
// (every probe mode with every object mode)
int obj_modes(const ptyr_geom& g) { return g.n_obj > 0 ? g.n_obj : 1; }
int chain_modes(const ptyr_geom& g) { return g.M * obj_modes(g); }

// the data terms of the loss: the loss_kind term alone at weight 1, or the
// weighted Gaussian and / or Poisson terms of Eq. 9
LossTerms loss_terms(const ptyr_geom& g) {
    LossTerms lt{};
    if (!(g.w_gaussian > 0.0) && !(g.w_poisson > 0.0)) {
        lt.n = 1;
        lt.k[0] = g.loss_kind;
        lt.p[0] = g.loss_p;
        lt.w[0] = 1.0;
        return lt;
    }
    if (g.w_gaussian > 0.0) {
        lt.k[lt.n] = PTYR_LOSS_GAUSSIAN;
        lt.p[lt.n] = g.p_gaussian > 0.0 ? g.p_gaussian : 0.5;
        lt.w[lt.n++] = g.w_gaussian;
    }
    if (g.w_poisson > 0.0) {
        lt.k[lt.n] = PTYR_LOSS_POISSON;
        lt.p[lt.n] = g.p_poisson > 0.0 ? g.p_poisson : 1.0;
        lt.w[lt.n++] = g.w_poisson;
    }
    return lt;
}
// two data terms are folded into the weights once both batch factors are known
bool two_terms(const ptyr_geom& g) { return loss_terms(g).n > 1; }

struct Layout {
    size_t Oc, Phat, pinfo, Imode, Ibuf, wbuf, lpart, scal, spart, pac, err, store, gO, gPhat, gPsum, part, gamp, gphase,
        gprobe, gdz, gpos, gtilt, wave, cons, rzmat, kz, total, tab256;
    int keep, ckK, nck, waves_per_chain;
};

// Waves per chain that keep everything the gradient reads: 2S (phi_s, Y_s,
// far field) for the fused kernels, S + 1 for the N = 256 line passes (the
// wave entering each slice's row pass, far field).
size_t full_waves(const ptyr_geom* g) { return g->N == 256 ? (size_t)g->S + 1 : 2 * (size_t)g->S; }

// How the forward keeps waves under the budget (in waves of N x N complex
// per chain, B_max * M chains): all of them (full_waves) -> stride 1;
// else a 3-wave scratch plus checkpoints of phi every K >= 2 slices; with no
// room for a checkpoint, K = S + 1 (recompute from the probe).
void keep_plan(const ptyr_geom* g, int* keep, int* K, int* nck) {
    size_t per = (size_t)g->B_max * chain_modes(*g) * g->N * g->N * sizeof(float2);
    size_t fit = g->wave_budget_bytes / per;
    if (fit >= full_waves(g)) { *keep = KEEP_FULL; *K = 1; *nck = 0; return; }
    *keep = KEEP_CKPT;
    size_t avail = fit > 3 ? fit - 3 : 0;
    if (avail == 0) { *K = g->S + 1; *nck = 0; return; }
    int k = std::max(2, (int)((g->S + avail - 1) / avail));
    while ((size_t)((g->S + k - 1) / k) > avail) ++k;
    *K = k;
    *nck = (g->S + k - 1) / k;
}

int checkpoint_stride(const ptyr_geom* g) {
    int keep, K, nck;
    keep_plan(g, &keep, &K, &nck);
    return K;
}

Layout make_layout(const ptyr_geom* g) {
    Layout L;
    const size_t NN = (size_t)g->N * g->N, HW = (size_t)g->H * g->W, B = g->B_max, M = g->M, S = g->S;
    const size_t Mc = chain_modes(*g), OS = obj_modes(*g) * S;     // chain modes; object slices of all modes
    keep_plan(g, &L.keep, &L.ckK, &L.nck);
    L.waves_per_chain = L.keep == KEEP_FULL ? (int)full_waves(g) : L.nck + 3;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    L.Oc = take(OS * HW * sizeof(float2));
    L.Phat = take(M * NN * sizeof(float2));
    L.pinfo = take(B * sizeof(PosInfo));
    L.Imode = take(B * Mc * NN * sizeof(float));
    L.Ibuf = take(B * NN * sizeof(float));
    L.wbuf = take(B * NN * sizeof(float));
    L.lpart = take(2 * NLP * NPART * sizeof(double));   // one block of NPART per row range
    L.scal = take(8 * sizeof(double));
    L.spart = take(B * OS * sizeof(double));           // sparsity-term partial sums
    L.pac = take(2 * NN * sizeof(double) + PAC_BLOCKS * sizeof(double));   // PACBED R, Abar; partial sums
    L.err = take(sizeof(int));
    L.store = take(B * Mc * (size_t)L.waves_per_chain * NN * sizeof(float2));
    L.gO = take(B * Mc * S * NN * sizeof(float2));
    L.gPhat = take(B * Mc * NN * sizeof(float2));
    L.gPsum = take(M * NN * sizeof(float2));
    L.part = take(B * Mc * (g->N == 256 ? NBLK256 : 1) * 8 * sizeof(double));
    L.gamp = take(OS * HW * sizeof(float));
    L.gphase = take(OS * HW * sizeof(float));
    L.gprobe = take(M * NN * sizeof(float2));
    L.gdz = take(sizeof(float));
    L.gpos = take((size_t)std::max(g->n_scan, 1) * 2 * sizeof(float));
    L.gtilt = take((size_t)std::max(g->n_scan, 1) * 2 * sizeof(float));
    L.wave = take(g->N == 256 ? B * Mc * NN * sizeof(float2) : 0);
    L.tab256 = take(g->N == 256 ? N256 * sizeof(float4) + B * sizeof(PosTab256) : 0);   // N = 256 pass factors
    // probe orthogonalisation: partial overlap sums (double complex), mixing
    // matrix (float complex), eigenvalues
    L.cons = take((size_t)ORTH_MAX_M * (ORTH_MAX_M + 1) / 2 * GRAM_MAX_CHUNKS * sizeof(cd) +
                  (size_t)ORTH_MAX_M * ORTH_MAX_M * sizeof(float2) + ORTH_MAX_M * sizeof(double));
    L.rzmat = take((size_t)RZ_REG_S * RZ_REG_S * sizeof(float));     // depth-filter matrix
    L.kz = take((S * HW + g->W + g->H + S) * sizeof(float2));       // k_z filter: the complex field, twiddles
    L.total = o;
    return L;
}

int grid_for(size_t n, int block = 256, int cap = 8192) {
    size_t g = (n + block - 1) / block;
    return (int)std::max<size_t>(1, std::min<size_t>(g, cap));
}

}  // namespace

struct ptyr_ctx {
    ptyr_geom g;
    char* ws;
    size_t ws_bytes;
    hipStream_t stream;
    // second stream for the other row range of a split batch, with the
    // fork / join events that order it against `stream` (default priority)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_mid = nullptr, ev_a1 = nullptr, ev_loss = nullptr, ev_sgrad = nullptr,
               ev_gdone = nullptr, ev_join = nullptr;
    int n_cu = 0;
    Layout L;
    int fwd_valid;   // waves / intensities of the last forward are in the workspace
    int fwd_B;
    int step_grads_clear = 0;   // ptyr_step's gradient buffers are all zero
    // instrumentation: event pairs around the fused kernels
    int timing = 0;
    int timing_err = 0;              // an event record failed since timing was last enabled
    std::vector<hipEvent_t> ev;      // 2 per launch
    std::vector<int> ev_kind;
    int ev_used = 0;
};

namespace {
constexpr int MAX_TIMED = 4096;
// A failed event record marks the launch untimed and is reported by the next
// ptyr_timing_read as PTYR_E_DEVICE.  Bound (bind = true): the caller launches
// one kernel with start() and stop() as that dispatch's own start and stop
// events (hipExtLaunchKernel), so no marker packet goes on the stream (the
// marker pairs cost the two-stream step about 1.6 %, bound events about 1.2 %).
struct TimedLaunch {
    ptyr_ctx* c;
    hipStream_t st;
    int slot;
    bool bound;
    TimedLaunch(ptyr_ctx* cc, int kind, hipStream_t s, bool bind = false) : c(cc), st(s), slot(-1), bound(bind) {
        if (c->timing && c->ev_used < MAX_TIMED) {
            slot = c->ev_used++;
            c->ev_kind[slot] = kind;
            if (!bound && hipEventRecord(c->ev[2 * slot], st) != hipSuccess) {
                c->ev_kind[slot] = -1;
                c->timing_err = 1;
                slot = -1;
            }
        }
    }
    hipEvent_t start() const { return slot >= 0 ? c->ev[2 * slot] : nullptr; }
    hipEvent_t stop() const { return slot >= 0 ? c->ev[2 * slot + 1] : nullptr; }
    ~TimedLaunch() {
        if (slot >= 0 && !bound && hipEventRecord(c->ev[2 * slot + 1], st) != hipSuccess) {
            c->ev_kind[slot] = -1;
            c->timing_err = 1;
        }
    }
};
}  // namespace

template <typename T> static T* at(ptyr_ctx* c, size_t off) { return reinterpret_cast<T*>(c->ws + off); }

extern "C" {

const char* ptyr_status_str(ptyr_status s) {
    switch (s) {
        case PTYR_OK: return "ok";
        case PTYR_E_ARG: return "invalid argument";
        case PTYR_E_BOUNDS: return "a probe patch leaves the object";
        case PTYR_E_NOMEM: return "workspace too small";
        case PTYR_E_DEVICE: return "HIP device error";
        case PTYR_E_NONFINITE: return "non-finite value in the loss inputs";
    }
    return "unknown status";
}

ptyr_status ptyr_check_geom(const ptyr_geom* g) {
    if (!g) return PTYR_E_ARG;
    if (g->N != 64 && g->N != 128 && g->N != 256) return PTYR_E_ARG;
    if (g->M < 1 || g->S < 1 || g->B_max < 1) return PTYR_E_ARG;
    if (g->H < g->N || g->W < g->N) return PTYR_E_ARG;
    if (!(g->dx > 0.0) || !(g->lambda > 0.0)) return PTYR_E_ARG;
    if (g->loss_kind != PTYR_LOSS_GAUSSIAN && g->loss_kind != PTYR_LOSS_POISSON) return PTYR_E_ARG;
    if (!(g->loss_p > 0.0) || !isfinite(g->loss_p)) return PTYR_E_ARG;
    if (g->flags & ~(PTYR_GLOBAL_TILT | PTYR_CHECK_FINITE)) return PTYR_E_ARG;
    // grid and index limits of the kernels
    if (g->n_obj < 0 || g->n_obj > 64) return PTYR_E_ARG;
    if ((double)g->B_max * g->M * (g->n_obj > 0 ? g->n_obj : 1) > 2147483647.0 / 2) return PTYR_E_ARG;
    // object elements (all modes and slices) at most 2^40: keeps every byte
    // count of the workspace layout far from size_t overflow
    if ((double)g->S * (g->n_obj > 0 ? g->n_obj : 1) * g->H * g->W > 1099511627776.0) return PTYR_E_ARG;
    if (g->n_scan < 0) return PTYR_E_ARG;
    if (!(g->sparse_w >= 0.0) || !isfinite(g->sparse_w)) return PTYR_E_ARG;
    if (!(g->pacbed_w >= 0.0) || !isfinite(g->pacbed_w)) return PTYR_E_ARG;
    for (double v : {g->w_gaussian, g->w_poisson, g->p_gaussian, g->p_poisson})
        if (!(v >= 0.0) || !isfinite(v)) return PTYR_E_ARG;
    if (g->N == 256) {   // the line-pass path keeps every wave (no recomputation)
        int keep, K, nck;
        keep_plan(g, &keep, &K, &nck);
        if (keep != KEEP_FULL) return PTYR_E_ARG;
    }
    return PTYR_OK;
}

ptyr_status ptyr_check_args(const ptyr_geom* g, int B, const float* pos_host) {
    ptyr_status st = ptyr_check_geom(g);
    if (st != PTYR_OK) return st;
    if (B < 1 || B > g->B_max) return PTYR_E_ARG;
    if (pos_host) {
        for (int j = 0; j < B; ++j) {
            float py = pos_host[2 * j], px = pos_host[2 * j + 1];
            if (!isfinite(py) || !isfinite(px)) return PTYR_E_BOUNDS;
            float ry = rintf(py), rx = rintf(px), half = (float)(g->N / 2);
            if (ry - half < 0.f || rx - half < 0.f || ry + half > (float)g->H || rx + half > (float)g->W)
                return PTYR_E_BOUNDS;
        }
    }
    return PTYR_OK;
}

size_t ptyr_workspace_bytes(const ptyr_geom* g) {
    if (ptyr_check_geom(g) != PTYR_OK) return 0;
    return make_layout(g).total;
}

ptyr_status ptyr_checkpoint_plan(const ptyr_geom* g, int* stride) {
    ptyr_status st = ptyr_check_geom(g);
    if (st != PTYR_OK) return st;
    if (!stride) return PTYR_E_ARG;
    *stride = checkpoint_stride(g);
    return PTYR_OK;
}

ptyr_status ptyr_create(const ptyr_geom* g, void* workspace, size_t ws_bytes, void* stream, ptyr_ctx** out) {
    ptyr_status st = ptyr_check_geom(g);
    if (st != PTYR_OK) return st;
    if (!out || !workspace) return PTYR_E_ARG;
    Layout L = make_layout(g);
    if (ws_bytes < L.total) return PTYR_E_NOMEM;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return PTYR_E_ARG;
    ptyr_ctx* c = new (std::nothrow) ptyr_ctx;
    if (!c) return PTYR_E_NOMEM;
    c->g = *g;
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = ws_bytes;
    c->stream = static_cast<hipStream_t>(stream);
    c->L = L;
    c->fwd_valid = 0;
    c->fwd_B = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_mid, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_loss, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_a1, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_sgrad, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_gdone, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)ptyr_destroy(c);
        return PTYR_E_DEVICE;
    }
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, c->stream, at<float>(c, L.err), (size_t)1);
    if (hipGetLastError() != hipSuccess) { (void)ptyr_destroy(c); return PTYR_E_DEVICE; }
    *out = c;
    return PTYR_OK;
}

ptyr_status ptyr_destroy(ptyr_ctx* ctx) {
    if (!ctx) return PTYR_E_ARG;
    bool ok = true;
    auto check = [&](hipError_t e) { ok = ok && e == hipSuccess; };
    if (ctx->side) check(hipStreamSynchronize(ctx->side));
    for (hipEvent_t e : ctx->ev)
        if (e) check(hipEventDestroy(e));
    for (hipEvent_t e : {ctx->ev_fork, ctx->ev_mid, ctx->ev_loss, ctx->ev_a1, ctx->ev_sgrad, ctx->ev_gdone,
                         ctx->ev_join})
        if (e) check(hipEventDestroy(e));
    if (ctx->side) check(hipStreamDestroy(ctx->side));
    delete ctx;
    return ok ? PTYR_OK : PTYR_E_DEVICE;
}

ptyr_status ptyr_timing_enable(ptyr_ctx* c, int on) {
    if (!c) return PTYR_E_ARG;
    if (on && c->ev.empty()) {
        c->ev.resize(2 * MAX_TIMED);
        c->ev_kind.assign(MAX_TIMED, -1);
        for (auto& e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                e = nullptr;
                return PTYR_E_DEVICE;
            }
    }
    c->timing = on ? 1 : 0;
    c->ev_used = 0;
    c->timing_err = 0;
    return PTYR_OK;
}

ptyr_status ptyr_timing_read(ptyr_ctx* c, int which, double* total_ms, int* launches) {
    if (!c || !total_ms || !launches) return PTYR_E_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipStreamSynchronize(c->side) != hipSuccess)
        return PTYR_E_DEVICE;
    double tot = 0.0;
    int n = 0;
    for (int i = 0; i < c->ev_used; ++i) {
        if (c->ev_kind[i] != which) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) return PTYR_E_DEVICE;
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return c->timing_err ? PTYR_E_DEVICE : PTYR_OK;
}

ptyr_status ptyr_sync(ptyr_ctx* ctx) {
    if (!ctx) return PTYR_E_ARG;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PTYR_E_DEVICE;
    int e = 0;
    if (hipMemcpy(&e, at<int>(ctx, ctx->L.err), sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return PTYR_E_DEVICE;
    if (e) {
        int z = 0;
        if (hipMemcpy(at<int>(ctx, ctx->L.err), &z, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return PTYR_E_DEVICE;
    }
    if (e & ERR_BOUNDS) return PTYR_E_BOUNDS;
    if (e & ERR_NONFINITE) return PTYR_E_NONFINITE;
    if (e & (ERR_ZERO_MEAN | ERR_INDEX)) return PTYR_E_ARG;
    return PTYR_OK;
}

}  // extern "C"

namespace {

WaveArgs wave_args(ptyr_ctx* c, const float* tilt, const float* dz, int B) {
    const ptyr_geom& g = c->g;
    WaveArgs a;
    a.Oc = at<float2>(c, c->L.Oc);
    a.Phat = at<float2>(c, c->L.Phat);
    a.pinfo = at<PosInfo>(c, c->L.pinfo);
    a.tilt = tilt;
    a.dz = dz;
    a.store = at<float2>(c, c->L.store);
    a.keep = c->L.keep;
    a.ckK = c->L.ckK;
    a.nck = c->L.nck;
    a.B = B; a.M = chain_modes(g); a.S = g.S; a.H = g.H; a.W = g.W;
    a.Mp = g.M;
    a.ostride = (size_t)g.S * g.H * g.W;
    a.chain0 = 0;
    a.dx = g.dx;
    a.lam = g.lambda;
    a.global_tilt = (g.flags & PTYR_GLOBAL_TILT) ? 1 : 0;
    a.Imode = at<float>(c, c->L.Imode);
    a.wgt = at<float>(c, c->L.wbuf);
    a.gO = at<float2>(c, c->L.gO);
    a.gPhat = at<float2>(c, c->L.gPhat);
    a.part = at<double>(c, c->L.part);
    return a;
}

// the fused kernels over chains [c0, c0 + nc) (chain = row * M + mode) on stream st
template <int N> void launch_forward(ptyr_ctx* c, WaveArgs a, int c0, int nc, hipStream_t st) {
    TimedLaunch t(c, PTYR_K_FORWARD, st, true);
    a.chain0 = c0;
    if (a.keep == KEEP_FULL)
        hipExtLaunchKernelGGL((k_forward<N, KEEP_FULL>), dim3(nc), dim3(N * N / 16), 0, st, t.start(), t.stop(), 0, a);
    else
        hipExtLaunchKernelGGL((k_forward<N, KEEP_CKPT>), dim3(nc), dim3(N * N / 16), 0, st, t.start(), t.stop(), 0, a);
}
template <int N> void launch_gradient(ptyr_ctx* c, WaveArgs a, int c0, int nc, hipStream_t st) {
    TimedLaunch t(c, PTYR_K_GRADIENT, st, true);
    a.chain0 = c0;
    if (a.keep == KEEP_FULL)
        hipExtLaunchKernelGGL((k_gradient<N, KEEP_FULL>), dim3(nc), dim3(N * N / 16), 0, st, t.start(), t.stop(), 0, a);
    else
        hipExtLaunchKernelGGL((k_gradient<N, KEEP_CKPT>), dim3(nc), dim3(N * N / 16), 0, st, t.start(), t.stop(), 0,
                              a);
}
// N = 256: forward and gradient as line passes (lines256.hpp)
Pass256 pass256(ptyr_ctx* c, const WaveArgs& a, int s) {
    Pass256 P;
    P.a = a;
    P.wave = at<float2>(c, c->L.wave);
    P.tw = at<float4>(c, c->L.tab256);
    P.tab = reinterpret_cast<const PosTab256*>(at<float4>(c, c->L.tab256) + N256);
    P.s = s;
    P.mg = 1;
    return P;
}
// the passes' twiddles and per-position factors for the batch of a
void tables256(ptyr_ctx* c, const WaveArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k256_tables, dim3(a.B), dim3(256), 0, st, a, at<float4>(c, c->L.tab256),
                       reinterpret_cast<PosTab256*>(at<float4>(c, c->L.tab256) + N256));
}
// probe modes whose patch gradients the N = 256 gradient row pass sums per
// workgroup: the largest divisor of the probe modes up to 8 (measured at the
// 16-position, 8-mode batch: groups of 8, 4 and 2 give 6.65, 6.76 and
// 7.08 ms per step); 1 for N = 64 and 128
int row_group(const ptyr_geom& g) {
    if (g.N != 256) return 1;
    for (int d = 8; d > 1; --d)
        if (g.M % d == 0) return d;
    return 1;
}
void forward256(ptyr_ctx* c, WaveArgs a, int c0, int nc, hipStream_t st) {
    TimedLaunch t(c, PTYR_K_FORWARD, st);
    a.chain0 = c0;
    const dim3 grid(nc * NBLK256), blk(256);
    tables256(c, a, st);
    hipLaunchKernelGGL(k256_fwd_col, grid, blk, 0, st, pass256(c, a, -1));
    for (int s = 0; s < a.S; ++s) {
        hipLaunchKernelGGL(k256_fwd_row, grid, blk, 0, st, pass256(c, a, s));
        hipLaunchKernelGGL(k256_fwd_col, grid, blk, 0, st, pass256(c, a, s));
    }
}
void gradient256(ptyr_ctx* c, WaveArgs a, int c0, int nc, hipStream_t st) {
    TimedLaunch t(c, PTYR_K_GRADIENT, st);
    a.chain0 = c0;
    const dim3 grid(nc * NBLK256), blk(256);
    tables256(c, a, st);
    hipLaunchKernelGGL(k256_grad_col, grid, blk, 0, st, pass256(c, a, a.S));
    // the row pass takes row_group(g) chains per workgroup (c0 and nc are
    // multiples of it: N = 256 batches are not split)
    const int mg = row_group(c->g);
    const dim3 rgrid(nc / mg * NBLK256);
    for (int s = a.S - 1; s >= 0; --s) {
        Pass256 P = pass256(c, a, s);
        P.mg = mg;
        hipLaunchKernelGGL(k256_grad_row, rgrid, blk, 0, st, P);
        hipLaunchKernelGGL(k256_grad_col, grid, blk, 0, st, pass256(c, a, s));
    }
}
void forward_chains(ptyr_ctx* c, const WaveArgs& a, int c0, int nc, hipStream_t st) {
    if (c->g.N == 64) launch_forward<64>(c, a, c0, nc, st);
    else if (c->g.N == 128) launch_forward<128>(c, a, c0, nc, st);
    else forward256(c, a, c0, nc, st);
}
void gradient_chains(ptyr_ctx* c, const WaveArgs& a, int c0, int nc, hipStream_t st) {
    if (c->g.N == 64) launch_gradient<64>(c, a, c0, nc, st);
    else if (c->g.N == 128) launch_gradient<128>(c, a, c0, nc, st);
    else gradient256(c, a, c0, nc, st);
}

// probe transforms, positions and transmission in one launch; the streaming
// part gets about two workgroups per compute unit (the transform's LDS allows
// no more), four elements per thread at least
template <int N>
void launch_prepare(ptyr_ctx* c, const float* amp, const float* phase, const float* probe, const float* pos,
                    const int* idx, int n_rows, int B, size_t nobj, hipStream_t st, int distinct) {
    const ptyr_geom& g = c->g;
    constexpr int T = N * N / 16;
    const size_t want = (nobj + 4 * (size_t)T - 1) / (4 * (size_t)T);
    const int nb = (int)std::max<size_t>(1, std::min<size_t>(want, 2 * (size_t)std::max(c->n_cu, 1)));
    hipLaunchKernelGGL(k_prepare<N>, dim3(g.M + nb), dim3(T), 0, st, amp, phase, at<float2>(c, c->L.Oc), nobj, pos,
                       idx, idx ? n_rows : B, B, g.H, g.W, at<PosInfo>(c, c->L.pinfo), at<int>(c, c->L.err),
                       reinterpret_cast<const float2*>(probe), at<float2>(c, c->L.Phat), g.M, distinct);
}
template <int N> void launch_probe_ifft_acc(ptyr_ctx* c, float* g_probe, hipStream_t st) {
    hipLaunchKernelGGL((k_fft2<N, +1, true>), dim3(c->g.M), dim3(N * N / 16), 0, st,
                       at<float2>(c, c->L.gPsum), reinterpret_cast<float2*>(g_probe));
}

// Work shared by every row of a batch: transmission of all slices, validated
// positions, probe spectra.
void prepare_forward(ptyr_ctx* c, const float* amp, const float* phase, const float* probe, const float* pos,
                     const int* idx, int n_rows, int B, int distinct) {
    const hipStream_t st = c->stream;
    const ptyr_geom& g = c->g;
    size_t nobj = (size_t)obj_modes(g) * g.S * g.H * g.W;
    if (g.N == 64) launch_prepare<64>(c, amp, phase, probe, pos, idx, n_rows, B, nobj, st, distinct);
    else if (g.N == 128) launch_prepare<128>(c, amp, phase, probe, pos, idx, n_rows, B, nobj, st, distinct);
    else {
        hipLaunchKernelGGL(k_transmission, dim3(grid_for((nobj + 7) / 8)), dim3(256), 0, st, amp, phase,
                           at<float2>(c, c->L.Oc), nobj);
        hipLaunchKernelGGL(k_positions, dim3((B + 63) / 64), dim3(64), 0, st, pos, idx, idx ? n_rows : B, B, g.N,
                           g.H, g.W, at<PosInfo>(c, c->L.pinfo), at<int>(c, c->L.err), distinct);
        const dim3 grid(g.M * NBLK256), blk(256);
        hipLaunchKernelGGL((k256_fft<-1, true, false>), grid, blk, 0, st, reinterpret_cast<const float2*>(probe),
                           at<float2>(c, c->L.Phat));
        hipLaunchKernelGGL((k256_fft<-1, false, false>), grid, blk, 0, st, at<float2>(c, c->L.Phat),
                           at<float2>(c, c->L.Phat));
    }
}

void modesum_rows(ptyr_ctx* c, int r0, int nr, hipStream_t st) {
    const ptyr_geom& g = c->g;
    const size_t NN = (size_t)g.N * g.N;
    hipLaunchKernelGGL(k_modesum, dim3(grid_for((size_t)nr * NN)), dim3(256), 0, st,
                       at<float>(c, c->L.Imode) + (size_t)r0 * chain_modes(g) * NN,
                       at<float>(c, c->L.Ibuf) + (size_t)r0 * NN, nr, chain_modes(g), g.N);
}

ptyr_status run_forward(ptyr_ctx* c, const float* amp, const float* phase, const float* probe, const float* pos,
                        const float* tilt, const float* dz, const int* idx, int n_rows, int B) {
    prepare_forward(c, amp, phase, probe, pos, idx, n_rows, B, 0);
    forward_chains(c, wave_args(c, tilt, dz, B), 0, B * chain_modes(c->g), c->stream);
    modesum_rows(c, 0, B, c->stream);
    if (hipGetLastError() != hipSuccess) return PTYR_E_DEVICE;
    c->fwd_valid = 1;
    c->fwd_B = B;
    return PTYR_OK;
}

// Mode sum, loss partial sums (into partial-sum range `slot` of NPART
// blocks, so that the final pass adds ranges in a fixed order) and unscaled
// gradient weights of rows [r0, r0 + nr).  nm: measured patterns addressable
// through midx, or the batch size without it.
void loss_rows(ptyr_ctx* c, const float* Ie, const int* midx, int nm, int r0, int nr, int slot, hipStream_t st) {
    const ptyr_geom& g = c->g;
    const size_t NN = (size_t)g.N * g.N;
    hipLaunchKernelGGL(k_loss_rows, dim3(NPART), dim3(256), 0, st,
                       at<float>(c, c->L.Imode) + (size_t)r0 * chain_modes(g) * NN, at<float>(c, c->L.Ibuf) + (size_t)r0 * NN,
                       Ie, midx ? midx + r0 : nullptr, nm, nr, chain_modes(g), g.N,
                       loss_terms(g), r0, at<double>(c, c->L.lpart) + NLP * (size_t)slot * NPART,
                       at<float>(c, c->L.wbuf) + (size_t)r0 * NN, at<int>(c, c->L.err));
}

// Device buffers of the loss passes: partial sums (NLP per block, one range
// of NPART blocks per row range), batch scalars (8 doubles), PACBED buffers
// (2 N^2 + PAC_BLOCKS doubles), the error flag, and the sparsity partial sums
// (nullable).  A context takes them from its workspace; ptyr_loss_noalloc
// from the library's static device scratch.
struct LossBufs {
    double* lpart;
    double* scal;
    double* pac;
    int* err;
    const double* spart;
};
LossBufs loss_bufs(ptyr_ctx* c) {
    return LossBufs{at<double>(c, c->L.lpart), at<double>(c, c->L.scal), at<double>(c, c->L.pac),
                    at<int>(c, c->L.err), at<double>(c, c->L.spart)};
}

// with_sparse: add the sparsity term of the batch (its partial sums come
// from k_sparse_partial) to the loss
void loss_final_with(const ptyr_geom& g, const LossBufs& b, int nslots, int B, double* loss_dev, hipStream_t st,
                     bool with_sparse) {
    const double n = (double)B * g.N * g.N;
    const bool sp = with_sparse && g.sparse_w > 0.0 && b.spart;
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, b.lpart, nslots * NPART, n, loss_terms(g),
                       (g.flags & PTYR_CHECK_FINITE) ? 1 : 0, b.scal, loss_dev, b.err, b.spart,
                       sp ? B * g.S * obj_modes(g) : 0,
                       sp ? g.sparse_w / ((double)B * g.S * obj_modes(g) * g.N * g.N) : 0.0);
}
void loss_final(ptyr_ctx* c, int nslots, int B, double* loss_dev, hipStream_t st, bool with_sparse) {
    loss_final_with(c->g, loss_bufs(c), nslots, B, loss_dev, st, with_sparse);
}

// PACBED term of a batch (after loss_final): adds it to the loss and its
// gradient to `out` (fold: the adjoint's unscaled weights, which then carry
// the data term's batch factor too; else ptyr_loss's dL/dI).
void pacbed_with(const ptyr_geom& g, const LossBufs& b, const float* I, const float* Ie, const int* midx,
                 int n_meas, int row0, int B, double* loss_dev, float* out, bool fold, hipStream_t st) {
    const int NN = g.N * g.N;
    double* pac = b.pac;
    double* part = pac + 2 * NN;
    const double p = loss_terms(g).p[0];           // the first data term's power (its normaliser is scal[2])
    hipLaunchKernelGGL(k_pacbed_partial, dim3(PAC_BLOCKS), dim3(256), 0, st, I, Ie, midx, n_meas, row0, B, NN,
                       p, pac, part);
    hipLaunchKernelGGL(k_pacbed_final, dim3(1), dim3(64), 0, st, part, PAC_BLOCKS, NN, B, p, g.pacbed_w, b.scal,
                       loss_dev, fold ? 1 : 0);
    if (out)
        hipLaunchKernelGGL(k_pacbed_grad, dim3(grid_for((size_t)B * NN)), dim3(256), 0, st, out, B, g.N, p, pac,
                           b.scal, fold ? 1 : 0, fold ? 2.f : 1.f, fold ? 1 : 0);
}
void pacbed(ptyr_ctx* c, const float* I, const float* Ie, const int* midx, int n_meas, int row0, int B,
            double* loss_dev, float* out, bool fold, hipStream_t st) {
    pacbed_with(c->g, loss_bufs(c), I, Ie, midx, n_meas, row0, B, loss_dev, out, fold, st);
}

// ptyr_loss on explicit buffers: partial sums, final pass, dL/dI, PACBED term
ptyr_status loss_pass(const ptyr_geom& g, const LossBufs& b, const float* Im, const float* Ie, const int* midx,
                      int n_meas, int B, double* loss_dev, float* dLdI, hipStream_t st) {
    const int NN = g.N * g.N;
    const size_t n = (size_t)B * NN;
    const int nm = midx ? n_meas : B;
    hipLaunchKernelGGL(k_loss_partial, dim3(NPART), dim3(256), 0, st, Im, Ie, midx, nm, B, NN, loss_terms(g),
                       b.lpart, b.err);
    loss_final_with(g, b, 1, B, loss_dev, st, false);
    if (dLdI)
        hipLaunchKernelGGL(k_loss_grad, dim3(grid_for(n)), dim3(256), 0, st, Im, Ie, midx, nm, B, g.N,
                           loss_terms(g), b.scal, dLdI);
    if (g.pacbed_w > 0.0) pacbed_with(g, b, Im, Ie, midx, nm, 0, B, loss_dev, dLdI, false, st);
    return hipGetLastError() == hipSuccess ? PTYR_OK : PTYR_E_DEVICE;
}

ptyr_status run_loss(ptyr_ctx* c, const float* Im, const float* Ie, const int* midx, int n_meas, int B,
                     double* loss_dev, float* dLdI) {
    return loss_pass(c->g, loss_bufs(c), Im, Ie, midx, n_meas, B, loss_dev, dLdI, c->stream);
}

// ------------------------------------------------------------------ allocation-free loss
// The scratch of ptyr_loss_noalloc: one set of loss buffers (LossBufs) for
// any N <= 256, in a file-scope device array (each device holds its own copy
// until the process ends).  Host code never uses the array's name as an
// address: its device address is looked up once per device.
constexpr size_t NOALLOC_PART = (size_t)NLP * NPART;                   // doubles
constexpr size_t NOALLOC_SCAL = 8;
constexpr size_t NOALLOC_PAC = 2 * 256 * 256 + PAC_BLOCKS;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_PART + NOALLOC_SCAL + NOALLOC_PAC;
static_assert(NOALLOC_DOUBLES * sizeof(double) == PTYR_NOALLOC_SCRATCH_BYTES, "scratch size in ptyr.h");
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

static_assert(ERR_BOUNDS == PTYR_ERRBIT_BOUNDS && ERR_NONFINITE == PTYR_ERRBIT_NONFINITE &&
                  ERR_ZERO_MEAN == PTYR_ERRBIT_ZERO_MEAN && ERR_INDEX == PTYR_ERRBIT_INDEX,
              "error bits in ptyr.h");

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch_dev[MAX_DEVICES] = {};

// the current device's address of `scratch` (looked up on the first call on
// each device, with that device current)
ptyr_status scratch_address(double** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return PTYR_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PTYR_E_DEVICE;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return PTYR_OK;
}

// A batch of more chains (one workgroup each, one workgroup per compute unit)
// than the chip has compute units would leave part of the chip idle in the
// second round of each fused kernel.  It runs instead on two streams:
//   main: forward of chains [0, n_cu) (every compute unit busy); loss of the
//         rows wholly inside that range; gradient of as many of their chains
//         as compute units are left over (g1); later the gradient of chains
//         [n_cu, B*M) and the scatter of the remaining rows.
//   side: forward of chains [n_cu, B*M) as compute units free up; loss of the
//         remaining rows; gradient of chains [g1, n_cu); then the batch
//         factor and the object scatter of the first range's rows, in the
//         compute units the main stream's last gradient launch leaves free.
// Small kernels are issued only when compute units are free, so they are not
// queued behind pending workgroups.  Returns n_cu (0: no split).
int split_chains(const ptyr_ctx* c, int B) {
    const ptyr_geom& g = c->g;
    const int Mc = chain_modes(g);
    if (g.N > 128 || c->n_cu <= 0 || B * Mc <= c->n_cu || g.pacbed_w > 0.0 || two_terms(g)) return 0;
    return c->n_cu / Mc >= 1 ? c->n_cu : 0;
}

ptyr_status run_adjoint(ptyr_ctx* c, const float* amp, const float* phase, const float* probe, const float* pos,
                        const float* tilt, const float* dz, const int* idx, int n_rows, int B,
                        const float* I_meas, float* g_amp, float* g_phase, float* g_probe, float* g_pos,
                        float* g_tilt, float* g_dz, double* loss_dev, unsigned flags,
                        const ObjAdam* fuse = nullptr, const SegAdam* seg = nullptr) {
    const ptyr_geom& g = c->g;
    const int M = chain_modes(g), nm = idx ? n_rows : B, BM = B * M;   // M: chain modes
    const bool reuse = (flags & PTYR_REUSE_FORWARD) && c->fwd_valid && c->fwd_B == B;
    const int nA = reuse ? 0 : split_chains(c, B);
    const bool fold = g.pacbed_w > 0.0 || two_terms(g);     // weights finished before the gradient
    if (!reuse) prepare_forward(c, amp, phase, probe, pos, idx, n_rows, B, 1);
    else if (idx)
        hipLaunchKernelGGL(k_check_distinct, dim3(1), dim3(256), 0, c->stream, idx, B, at<PosInfo>(c, c->L.pinfo),
                           at<int>(c, c->L.err));
    // sparsity term: |phase| over the batch's patches, before any update of the phase
    const bool sparse = g.sparse_w > 0.0;
    if (sparse)
        hipLaunchKernelGGL(k_sparse_partial, dim3(B, g.S * obj_modes(g)), dim3(256), 0, c->stream, phase,
                           at<PosInfo>(c, c->L.pinfo), g.S * obj_modes(g), g.N, g.H, g.W, at<double>(c, c->L.spart));
    const float sp =
        sparse && g_phase ? (float)(g.sparse_w / ((double)B * g.S * obj_modes(g) * g.N * g.N)) : 0.f;
    const WaveArgs a = wave_args(c, tilt, dz, B);
    const double* scale = at<double>(c, c->L.scal) + 1;     // the batch factor of w (after loss_final)
    // object-gradient scatter of batch rows [j0, j1) on stream st; `last`
    // (the batch's final scatter) runs the fused object Adam when asked
    // rows [j0, j1); `last` fuses the object's Adam (ptyr_step), for which
    // j0 > 0 means rows [0, j0) were scattered into the gradient buffers first
    auto scatter = [&](int j0, int j1, hipStream_t st, bool last) {
        if (!(g_amp || g_phase)) return;
        const int ntiles = ((g.H + 31) / 32) * ((g.W + 31) / 32);
        const dim3 grid(ntiles, g.S * obj_modes(g));
        // patch gradients per position and object mode: one per group of
        // row_group(g) probe modes (the N = 256 row pass sums each group)
        const int mg = row_group(g), Mg = g.M / mg, Mcg = M / mg;
        const bool mb8 = Mg % 8 == 0;
        const float2* gO = at<float2>(c, c->L.gO);
        const PosInfo* pinfo = at<PosInfo>(c, c->L.pinfo);
        if (last && fuse) {
            ObjAdam ad = *fuse;
            ad.gin = j0 > 0 ? 1 : 0;
            if (mb8)
                hipLaunchKernelGGL((k_scatter_object<true, 8>), grid, dim3(256), 0, st, gO, pinfo, j0, j1, Mg, Mcg,
                                   g.S, g.N, g.H, g.W, amp, phase, scale, g_amp, g_phase, ad, sp);
            else
                hipLaunchKernelGGL((k_scatter_object<true, 4>), grid, dim3(256), 0, st, gO, pinfo, j0, j1, Mg, Mcg,
                                   g.S, g.N, g.H, g.W, amp, phase, scale, g_amp, g_phase, ad, sp);
        } else if (j1 > j0) {
            // the first scatter of a fused step writes its sums, any other adds them
            ObjAdam ad{};
            ad.assign = fuse && j0 == 0 ? 1 : 0;
            if (mb8)
                hipLaunchKernelGGL((k_scatter_object<false, 8>), grid, dim3(256), 0, st, gO, pinfo, j0, j1, Mg, Mcg,
                                   g.S, g.N, g.H, g.W, amp, phase, scale, g_amp, g_phase, ad, sp);
            else
                hipLaunchKernelGGL((k_scatter_object<false, 4>), grid, dim3(256), 0, st, gO, pinfo, j0, j1, Mg, Mcg,
                                   g.S, g.N, g.H, g.W, amp, phase, scale, g_amp, g_phase, ad, sp);
        }
    };
    // probe-spectrum sum and inverse transform, position / tilt / dz partials
    auto reductions = [&](hipStream_t st) {
        if (g_probe) {
            int NN = g.N * g.N;
            hipLaunchKernelGGL(k_sum_rows, dim3(grid_for((size_t)g.M * NN)), dim3(256), 0, st,
                               at<float2>(c, c->L.gPhat), at<float2>(c, c->L.gPsum), B * obj_modes(g), g.M, NN, scale);
            if (g.N == 64) launch_probe_ifft_acc<64>(c, g_probe, st);
            else if (g.N == 128) launch_probe_ifft_acc<128>(c, g_probe, st);
            else {
                const dim3 grid(g.M * NBLK256), blk(256);
                hipLaunchKernelGGL((k256_fft<+1, true, false>), grid, blk, 0, st, at<float2>(c, c->L.gPsum),
                                   at<float2>(c, c->L.gPsum));
                hipLaunchKernelGGL((k256_fft<+1, false, true>), grid, blk, 0, st, at<float2>(c, c->L.gPsum),
                                   reinterpret_cast<float2*>(g_probe));
            }
        }
        if (g_pos || g_tilt || g_dz)
            hipLaunchKernelGGL(k_param_grads, dim3(1), dim3(256), 0, st, at<double>(c, c->L.part),
                               g.N == 256 ? NBLK256 : 1, at<PosInfo>(c, c->L.pinfo), B, M, tilt, a.global_tilt, dz,
                               g.lambda, scale, g_pos, g_tilt, g_dz);
    };
    // ptyr_step: Adam of the probe, positions, tilts and dz, whose gradients
    // are complete once the reductions are; on the main stream right after
    // them, so it runs beside the last object scatter instead of after it
    auto seg_adam = [&]() {
        if (seg && seg->A.off[ADAM_SEGS] > 0)
            hipLaunchKernelGGL(k_adam_segs, dim3(grid_for(seg->A.off[ADAM_SEGS])), dim3(256), 0, c->stream, seg->A,
                               seg->b1, seg->b2, seg->eps, seg->bc1, seg->bc2s);
    };
    int scattered = 0;                                       // rows already scattered
    if (nA) {
        const int rA = nA / M;                                     // rows complete after the first forward
        const int g1 = std::min(rA * M, std::max(0, c->n_cu - (BM - nA)));   // early gradient chains
        if (hipEventRecord(c->ev_fork, c->stream) != hipSuccess ||
            hipStreamWaitEvent(c->side, c->ev_fork, 0) != hipSuccess)
            return PTYR_E_DEVICE;
        forward_chains(c, a, 0, nA, c->stream);
        forward_chains(c, a, nA, BM - nA, c->side);
        loss_rows(c, I_meas, idx, nm, 0, rA, 0, c->stream);
        // the side stream continues with the remaining rows once the first
        // range's forward and loss are done (its rows' weights are read by
        // the remaining gradient chains of the first range)
        if (hipEventRecord(c->ev_mid, c->stream) != hipSuccess ||
            hipStreamWaitEvent(c->side, c->ev_mid, 0) != hipSuccess)
            return PTYR_E_DEVICE;
        if (g1 > 0) gradient_chains(c, a, 0, g1, c->stream);
        loss_rows(c, I_meas, idx, nm, rA, B - rA, 1, c->side);
        if (hipEventRecord(c->ev_loss, c->side) != hipSuccess ||
            hipStreamWaitEvent(c->stream, c->ev_loss, 0) != hipSuccess)
            return PTYR_E_DEVICE;
        // main: the batch factor (both loss ranges are done) after its first
        // gradient launch, off the side stream's path to the scatter
        loss_final(c, 2, B, loss_dev, c->stream, true);
        if (hipEventRecord(c->ev_a1, c->stream) != hipSuccess) return PTYR_E_DEVICE;
        // side: the first range's remaining gradient chains, then (the first
        // gradient launch and the batch factor being done) the scatter of the
        // first range's complete rows, which runs in the compute units the
        // main stream's last gradient launch leaves free
        if (nA > g1) gradient_chains(c, a, g1, nA - g1, c->side);
        if (hipEventRecord(c->ev_sgrad, c->side) != hipSuccess ||
            hipStreamWaitEvent(c->side, c->ev_a1, 0) != hipSuccess)
            return PTYR_E_DEVICE;
        scatter(0, rA, c->side, false);
        // main: the second range's gradient chains, then (with the side
        // stream's chains done) the probe / parameter
        // reductions, which need every chain; the side stream meanwhile
        // scatters the remaining rows.  (The reductions' probe transform
        // needs whole compute units: issued first, on the stream that is
        // already running, it gets them before the scatter fills the chip.)
        gradient_chains(c, a, nA, BM - nA, c->stream);
        if (hipEventRecord(c->ev_gdone, c->stream) != hipSuccess ||
            hipStreamWaitEvent(c->side, c->ev_gdone, 0) != hipSuccess ||
            hipStreamWaitEvent(c->stream, c->ev_sgrad, 0) != hipSuccess)
            return PTYR_E_DEVICE;
        reductions(c->stream);
        seg_adam();
        scatter(rA, B, c->side, true);
        if (hipEventRecord(c->ev_join, c->side) != hipSuccess ||
            hipStreamWaitEvent(c->stream, c->ev_join, 0) != hipSuccess)
            return PTYR_E_DEVICE;
        scattered = B;
    } else {
        if (!reuse) forward_chains(c, a, 0, BM, c->stream);
        loss_rows(c, I_meas, idx, nm, 0, B, 0, c->stream);
        if (fold) {
            // the weights of two data terms and the PACBED weights need every
            // row's pattern and the batch factors before the gradient: fold
            // them into the weights
            loss_final(c, 1, B, loss_dev, c->stream, true);
            if (two_terms(g))
                hipLaunchKernelGGL(k_loss_mix, dim3(grid_for((size_t)B * g.N * g.N)), dim3(256), 0, c->stream,
                                   at<float>(c, c->L.wbuf), at<float>(c, c->L.Ibuf), I_meas, idx, nm, 0, B, g.N,
                                   loss_terms(g), at<double>(c, c->L.scal));
            if (g.pacbed_w > 0.0)
                pacbed(c, at<float>(c, c->L.Ibuf), I_meas, idx, nm, 0, B, loss_dev, at<float>(c, c->L.wbuf), true,
                       c->stream);
        }
        gradient_chains(c, a, 0, BM, c->stream);
    }
    c->fwd_valid = 1;
    c->fwd_B = B;
    if (!scattered) {
        if (!fold) loss_final(c, 1, B, loss_dev, c->stream, true);
        reductions(c->stream);
        seg_adam();
        scatter(0, B, c->stream, true);
    }
    return hipGetLastError() == hipSuccess ? PTYR_OK : PTYR_E_DEVICE;
}

void zero(ptyr_ctx* c, float* p, size_t n) {
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(256), 0, c->stream, p, n);
}


}  // namespace

extern "C" {

ptyr_status ptyr_forward(ptyr_ctx* c, const float* amp, const float* phase, const float* probe, const float* pos,
                         const float* tilt, const float* dz, const int* idx, int n_rows, int B, float* I_out) {
    if (!c) return PTYR_E_ARG;
    ptyr_status st = ptyr_check_args(&c->g, B, nullptr);
    if (st != PTYR_OK) return st;
    if (!amp || !phase || !probe || !pos || !tilt || !dz || !I_out) return PTYR_E_ARG;
    if (idx && n_rows < 1) return PTYR_E_ARG;
    st = run_forward(c, amp, phase, probe, pos, tilt, dz, idx, n_rows, B);
    if (st != PTYR_OK) return st;
    size_t n = (size_t)B * c->g.N * c->g.N;
    if (hipMemcpyAsync(I_out, at<float>(c, c->L.Ibuf), n * sizeof(float), hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
        return PTYR_E_DEVICE;
    return PTYR_OK;
}

ptyr_status ptyr_loss(ptyr_ctx* c, const float* I_model, const float* I_meas, const int* meas_idx, int n_meas,
                      int B, double* loss_dev, float* dLdI) {
    if (!c) return PTYR_E_ARG;
    ptyr_status st = ptyr_check_args(&c->g, B, nullptr);
    if (st != PTYR_OK) return st;
    if (!I_model || !I_meas || !loss_dev) return PTYR_E_ARG;
    if (meas_idx && n_meas < 1) return PTYR_E_ARG;
    return run_loss(c, I_model, I_meas, meas_idx, n_meas, B, loss_dev, dLdI);
}

ptyr_status ptyr_loss_noalloc(const ptyr_geom* g, const float* I_model, const float* I_meas, const int* meas_idx,
                              int n_meas, int B, double* loss_dev, float* dLdI, int* err_dev, void* stream) {
    ptyr_status st = ptyr_check_geom(g);
    if (st != PTYR_OK) return st;
    if (B < 1 || !I_model || !I_meas || !loss_dev || !err_dev) return PTYR_E_ARG;
    if (meas_idx && n_meas < 1) return PTYR_E_ARG;
    const size_t NN = (size_t)g->N * g->N;
    if (NOALLOC_PART + NOALLOC_SCAL + 2 * NN + PAC_BLOCKS > NOALLOC_DOUBLES) return PTYR_E_NOMEM;
    double* base = nullptr;
    st = scratch_address(&base);
    if (st != PTYR_OK) return st;
    // every buffer is written before it is read (partial sums by all NPART
    // blocks, scalars by the final pass, PACBED sums by its first pass), so
    // what an earlier call left needs no clearing
    const LossBufs b{base, base + NOALLOC_PART, base + NOALLOC_PART + NOALLOC_SCAL, err_dev, nullptr};
    return loss_pass(*g, b, I_model, I_meas, meas_idx, n_meas, B, loss_dev, dLdI,
                     static_cast<hipStream_t>(stream));
}

ptyr_status ptyr_adjoint(ptyr_ctx* c, const float* amp, const float* phase, const float* probe, const float* pos,
                         const float* tilt, const float* dz, const int* idx, int n_rows, int B,
                         const float* I_meas, float* g_amp, float* g_phase, float* g_probe, float* g_pos,
                         float* g_tilt, float* g_dz, double* loss_dev, unsigned flags) {
    if (!c) return PTYR_E_ARG;
    ptyr_status st = ptyr_check_args(&c->g, B, nullptr);
    if (st != PTYR_OK) return st;
    if (!amp || !phase || !probe || !pos || !tilt || !dz || !I_meas) return PTYR_E_ARG;
    if (flags & ~PTYR_REUSE_FORWARD) return PTYR_E_ARG;
    if (idx && n_rows < 1) return PTYR_E_ARG;
    return run_adjoint(c, amp, phase, probe, pos, tilt, dz, idx, n_rows, B, I_meas, g_amp, g_phase, g_probe, g_pos,
                       g_tilt, g_dz, loss_dev, flags);
}

ptyr_status ptyr_constrain(ptyr_ctx* c, float* amp, float* phase, float* probe, const ptyr_constraints* cfg) {
    if (!c || !cfg) return PTYR_E_ARG;
    const ptyr_geom& g = c->g;
    const bool rz = cfg->rz_sigma > 0.f;
    if (!(cfg->rz_sigma >= 0.f && cfg->rz_sigma <= 16.f)) return PTYR_E_ARG;
    if (rz && (!amp || !phase || g.S > RZ_MAX_S)) return PTYR_E_ARG;
    if (cfg->phase_positive && !phase) return PTYR_E_ARG;
    if (cfg->probe_orthogonal && (!probe || g.M > ORTH_MAX_M)) return PTYR_E_ARG;
    const bool kz = cfg->kz_beta > 0.f || cfg->kz_alpha > 0.f;
    int rad[3][32], nrad[3] = {0, 0, 0};
    if (!(cfg->kz_beta >= 0.f) || !(cfg->kz_alpha >= 0.f) || !isfinite(cfg->kz_beta) || !isfinite(cfg->kz_alpha))
        return PTYR_E_ARG;
    if (kz) {
        if (!amp || !phase || !(cfg->kz_dz > 0.f) || !isfinite(cfg->kz_dz)) return PTYR_E_ARG;
        if (std::max(g.S, std::max(g.H, g.W)) > KZ_MAX_SIDE) return PTYR_E_ARG;
        nrad[0] = fft_radices(g.W, rad[0]);
        nrad[1] = fft_radices(g.H, rad[1]);
        nrad[2] = fft_radices(g.S, rad[2]);
        if (nrad[0] < 0 || nrad[1] < 0 || nrad[2] < 0) return PTYR_E_ARG;
    }
    const hipStream_t st = c->stream;
    const size_t HW = (size_t)g.H * g.W;
    const int nob = obj_modes(g);
    // every object mode is filtered on its own (S x H x W each)
    for (int ob = 0; ob < nob; ++ob) {
        float* const amp_o = amp ? amp + (size_t)ob * g.S * HW : nullptr;
        float* const phase_o = phase ? phase + (size_t)ob * g.S * HW : nullptr;
        if (kz) {
            // amplitude + i phase: forward x and y passes, the z pass (forward,
            // weight, inverse), inverse y and x passes
            float2* zb = at<float2>(c, c->L.kz);
            float2* twx = zb + (size_t)g.S * HW;           // twiddle tables of the three line lengths
            float2* twy = twx + g.W;
            float2* twz = twy + g.H;
            hipLaunchKernelGGL(k_kz_twiddles, dim3(grid_for(g.W)), dim3(256), 0, st, twx, g.W);
            hipLaunchKernelGGL(k_kz_twiddles, dim3(grid_for(g.H)), dim3(256), 0, st, twy, g.H);
            hipLaunchKernelGGL(k_kz_twiddles, dim3(grid_for(g.S)), dim3(256), 0, st, twz, g.S);
            int gx, gy, gz;
            const KzPass px = kz_pass(g.W, 1, g.S * g.H, 0, (size_t)g.W, 1, rad[0], nrad[0], 16, twx, &gx);
            const KzPass py = kz_pass(g.H, g.S, g.W, HW, 1, (size_t)g.W, rad[1], nrad[1], 16, twy, &gy);
            const KzPass pz = kz_pass(g.S, 1, g.H * g.W, 0, 1, HW, rad[2], nrad[2], 256, twz, &gz);
            const KzWeight kw{g.S, g.H, g.W, (double)cfg->kz_beta, (double)cfg->kz_alpha, g.dx, (double)cfg->kz_dz};
            const dim3 blk(KZ_THREADS);
            hipLaunchKernelGGL((k_kz_lines<KZ_IN_FIELDS, -1>), dim3(gx), blk, kz_lds_bytes(px), st, zb, amp_o, phase_o,
                               px, kw);
            hipLaunchKernelGGL((k_kz_lines<0, -1>), dim3(gy), blk, kz_lds_bytes(py), st, zb, amp_o, phase_o, py, kw);
            hipLaunchKernelGGL((k_kz_lines<KZ_FILTER, 0>), dim3(gz), blk, kz_lds_bytes(pz), st, zb, amp_o, phase_o, pz,
                               kw);
            hipLaunchKernelGGL((k_kz_lines<0, +1>), dim3(gy), blk, kz_lds_bytes(py), st, zb, amp_o, phase_o, py, kw);
            hipLaunchKernelGGL((k_kz_lines<KZ_OUT_FIELDS, +1>), dim3(gx), blk, kz_lds_bytes(px), st, zb, amp_o,
                               phase_o, px, kw);
        }
        if (rz && g.S > 1) {
            // taps in double, normalised, then rounded (the same on every call)
            RzTaps t;
            t.R = (int)ceil(4.0 * (double)cfg->rz_sigma);
            double w[2 * RZ_MAX_R + 1], sum = 0.0;
            for (int k = -t.R; k <= t.R; ++k) {
                w[k + t.R] = exp(-(double)k * k / (2.0 * (double)cfg->rz_sigma * cfg->rz_sigma));
                sum += w[k + t.R];
            }
            for (int k = 0; k <= 2 * t.R; ++k) t.w[k] = (float)(w[k] / sum);
            float* fields[2] = {amp_o, phase_o};
            if (g.S <= RZ_REG_S) {
                float* Bm = at<float>(c, c->L.rzmat);
                hipLaunchKernelGGL(k_rz_matrix, dim3((g.S * g.S + 255) / 256), dim3(256), 0, st, t, g.S, Bm);
                const bool vec4 = HW % 4 == 0 && reinterpret_cast<uintptr_t>(amp_o) % 16 == 0 &&
                                  reinterpret_cast<uintptr_t>(phase_o) % 16 == 0;
                // amplitude (grid row 0) and phase (row 1) in one launch
                const dim3 grid((unsigned)((HW / (vec4 ? 4 : 1) + 255) / 256), 2);
                const int pos = cfg->phase_positive ? 1 : 0;
                TimedLaunch tl(c, PTYR_K_RZ, st);
                if (vec4)
                    hipLaunchKernelGGL(k_rz_filter_reg4, grid, dim3(256), 0, st, fields[0], fields[1], g.S, HW, Bm, pos);
                else
                    hipLaunchKernelGGL(k_rz_filter_reg, grid, dim3(256), 0, st, fields[0], fields[1], g.S, HW, Bm, pos);
            } else {
                const int T = rz_threads(g.S);
                const dim3 grid((unsigned)((HW + T - 1) / T));
                const size_t lds = (size_t)g.S * T * sizeof(float);
                for (int f = 0; f < 2; ++f) {
                    TimedLaunch tl(c, PTYR_K_RZ, st);
                    hipLaunchKernelGGL(k_rz_filter, grid, dim3(T), lds, st, fields[f], g.S, HW, t,
                                       f == 1 && cfg->phase_positive ? 1 : 0);
                }
            }
        }
    }
    if (!(rz && g.S > 1) && cfg->phase_positive)
        hipLaunchKernelGGL(k_clip_negative, dim3(grid_for((size_t)nob * g.S * HW)), dim3(256), 0, st, phase,
                           (size_t)nob * g.S * HW);
    if (cfg->probe_orthogonal && g.M > 1) {
        const int M = g.M, NN = g.N * g.N, nchunk = (NN + GRAM_CHUNK - 1) / GRAM_CHUNK;
        cd* part = at<cd>(c, c->L.cons);
        float2* V = reinterpret_cast<float2*>(part + (size_t)ORTH_MAX_M * (ORTH_MAX_M + 1) / 2 * GRAM_MAX_CHUNKS);
        double* lam = reinterpret_cast<double*>(V + ORTH_MAX_M * ORTH_MAX_M);
        float2* P = reinterpret_cast<float2*>(probe);
        hipLaunchKernelGGL(k_probe_gram, dim3(nchunk, M * (M + 1) / 2), dim3(256), 0, st, P, M, NN, part);
        hipLaunchKernelGGL(k_probe_eig, dim3(1), dim3(64), 0, st, part, nchunk, M, V, lam);
        const size_t lds = ((size_t)M * 256 + (size_t)M * M) * sizeof(float2);
        hipLaunchKernelGGL(k_probe_mix, dim3((NN + 255) / 256), dim3(256), lds, st, P, M, NN, V);
    }
    return hipGetLastError() == hipSuccess ? PTYR_OK : PTYR_E_DEVICE;
}

ptyr_status ptyr_step(ptyr_ctx* c, ptyr_params* p, const int* idx, int B, const float* I_meas_all,
                      const ptyr_lr* lr, double* loss_dev) {
    if (!c || !p || !lr || !idx || !I_meas_all) return PTYR_E_ARG;
    ptyr_status st = ptyr_check_args(&c->g, B, nullptr);
    if (st != PTYR_OK) return st;
    if (!p->amp || !p->phase || !p->probe || !p->pos || !p->tilt || !p->dz) return PTYR_E_ARG;
    if (p->n_pos < B || p->n_pos > c->g.n_scan) return PTYR_E_ARG;
    const float rates[6] = {lr->amp, lr->phase, lr->probe, lr->pos, lr->tilt, lr->dz};
    float* const mv[6][2] = {{p->m_amp, p->v_amp}, {p->m_phase, p->v_phase}, {p->m_probe, p->v_probe},
                             {p->m_pos, p->v_pos}, {p->m_tilt, p->v_tilt}, {p->m_dz, p->v_dz}};
    for (int k = 0; k < 6; ++k) {
        if (!(rates[k] >= 0.f) || !isfinite(rates[k])) return PTYR_E_ARG;
        if (rates[k] > 0.f && (!mv[k][0] || !mv[k][1])) return PTYR_E_ARG;
    }
    if (!(lr->beta1 >= 0.f && lr->beta1 < 1.f && lr->beta2 >= 0.f && lr->beta2 < 1.f && lr->eps >= 0.f))
        return PTYR_E_ARG;
    const ptyr_geom& g = c->g;
    const bool gt = (g.flags & PTYR_GLOBAL_TILT) != 0;
    const size_t nobj = (size_t)obj_modes(g) * g.S * g.H * g.W, nprb = (size_t)g.M * g.N * g.N * 2;
    const size_t npos = (size_t)p->n_pos * 2, ntilt = gt ? 2 : npos;
    float* gamp = at<float>(c, c->L.gamp);
    float* gphase = at<float>(c, c->L.gphase);
    float* gprobe = at<float>(c, c->L.gprobe);
    float* gdz = at<float>(c, c->L.gdz);
    float* gpos = at<float>(c, c->L.gpos);
    float* gtilt = at<float>(c, c->L.gtilt);
    // The six gradient buffers are consecutive in the workspace; they are
    // cleared once here and afterwards by each step's Adam as it reads them
    // (an interrupted step leaves them to be cleared again).  The object's two
    // need no clearing: only the first scatter of a two-stream batch writes
    // them (its sums, on the tiles its rows touch), and the fused Adam reads
    // exactly those tiles.
    if (!c->step_grads_clear)
        zero(c, gamp, (size_t)(reinterpret_cast<char*>(at<float>(c, c->L.gtilt) + std::max(g.n_scan, 1) * 2) -
                               reinterpret_cast<char*>(gamp)) / sizeof(float));
    c->step_grads_clear = 0;
    const int64_t t = p->step + 1;
    const double bc1 = 1.0 - pow((double)lr->beta1, (double)t);
    const double bc2 = 1.0 - pow((double)lr->beta2, (double)t);
    // the object's Adam runs inside the batch's last object scatter
    const ObjAdam oa{p->amp,     p->phase,  p->m_amp,   p->v_amp,  p->m_phase,    p->v_phase,
                     rates[0],   rates[1],  lr->beta1,  lr->beta2, lr->eps,       (float)bc1,
                     (float)sqrt(bc2), 0};
    SegAdam sa;
    {
        AdamSegs& A = sa.A;
        float* const params[6] = {p->amp, p->phase, p->probe, p->pos, p->tilt, p->dz};
        float* const grads[6] = {gamp, gphase, gprobe, gpos, gtilt, gdz};
        const size_t sizes[6] = {nobj, nobj, nprb, npos, ntilt, 1};
        A.off[0] = 0;
        for (int k = 0; k < 6; ++k) {
            // a zero rate leaves the parameter and its moments alone; the
            // object and probe gradients are then not even accumulated, the
            // position / tilt / dz ones are and only need clearing.  The
            // object (k < 2) was updated by the fused scatter.
            const bool on = rates[k] > 0.f && k >= 2;
            A.p[k] = params[k];
            A.g[k] = grads[k];
            A.m[k] = mv[k][0];
            A.v[k] = mv[k][1];
            A.lr[k] = rates[k];
            A.upd[k] = on ? 1 : 0;
            A.off[k + 1] = A.off[k] + ((on || k >= 3) ? sizes[k] : 0);
        }
        sa.b1 = lr->beta1;
        sa.b2 = lr->beta2;
        sa.eps = lr->eps;
        sa.bc1 = (float)bc1;
        sa.bc2s = (float)sqrt(bc2);
    }
    st = run_adjoint(c, p->amp, p->phase, p->probe, p->pos, p->tilt, p->dz, idx, p->n_pos, B, I_meas_all,
                     rates[0] > 0.f ? gamp : nullptr, rates[1] > 0.f ? gphase : nullptr,
                     rates[2] > 0.f ? gprobe : nullptr, gpos, gtilt, gdz, loss_dev, 0, &oa, &sa);
    if (st != PTYR_OK) return st;
    c->step_grads_clear = 1;
    p->step = t;
    return hipGetLastError() == hipSuccess ? PTYR_OK : PTYR_E_DEVICE;
}

}  // extern "C"
