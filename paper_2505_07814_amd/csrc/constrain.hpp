// constrain.hpp - per-iteration constraints on the object and probe (the
// paper's Sec. "Physical constraints"): the r_z depth filter with phase
// positivity, and probe-mode orthogonalisation.
#pragma once
#include <hip/hip_runtime.h>

namespace ptyr {

constexpr int RZ_MAX_R = 64;        // largest tap radius (rz_sigma <= 16)
constexpr int ORTH_MAX_M = 24;      // most probe modes the orthogonalisation takes
constexpr int RZ_MAX_S = 256;       // deepest stack the depth filter takes
constexpr int GRAM_CHUNK = 1024;    // pixels per partial overlap sum
constexpr int GRAM_MAX_CHUNKS = 64; // N = 256: 65536 / 1024

struct RzTaps {
    float w[2 * RZ_MAX_R + 1];      // normalised taps w[k + R], k = -R..R
    int R;
};

// index i of a stack of S slices extended by mirroring about its outer faces
__device__ __forceinline__ int mirror_slice(int i, int S) {
    if (i >= 0 && i < S) return i;                       // inside, or one reflection (taps within S)
    if (i < 0 && i >= -S) return -1 - i;
    if (i >= S && i < 2 * S) return 2 * S - 1 - i;
    if (S == 1) return 0;
    const int period = 2 * S;
    i %= period;
    if (i < 0) i += period;
    return i < S ? i : period - 1 - i;
}

// r_z filter of one field (S x HW, in place), then optionally max(., 0).
// A thread owns one pixel's column: it reads the S values (consecutive
// threads take consecutive pixels, so each slice is one coalesced row per
// wave) into its own LDS column, which serves as an indexable array, and
// writes the filtered column back.  A thread touches only its own column,
// so no barrier is needed.  Dynamic LDS: S * blockDim.x floats.
__global__ __launch_bounds__(256) void k_rz_filter(float* v, int S, size_t HW, RzTaps taps, int positive) {
    extern __shared__ float col[];
    const int T = blockDim.x;
    const size_t px = (size_t)blockIdx.x * T + threadIdx.x;
    if (px >= HW) return;
    float* c = col + threadIdx.x;
    int s = 0;
    for (; s + 4 <= S; s += 4) {               // four reads in flight per thread
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = v[(size_t)(s + u) * HW + px];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[(s + u) * T] = x[u];
    }
    for (; s < S; ++s) c[s * T] = v[(size_t)s * HW + px];
    const int R = taps.R;
    for (s = 0; s < S; ++s) {
        float acc = 0.f;
        for (int k = -R; k <= R; ++k) acc = fmaf(taps.w[k + R], c[mirror_slice(s + k, S) * T], acc);
        v[(size_t)s * HW + px] = positive ? fmaxf(acc, 0.f) : acc;
    }
}

// The depth filter as an S x S matrix: B[s][s'] = sum of the taps w_k with
// mirror(s + k) = s' (the mirrored boundary folded in).  One thread per entry.
__global__ void k_rz_matrix(RzTaps taps, int S, float* Bm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * S) return;
    const int s = i / S, s2 = i % S;
    float b = 0.f;
    for (int k = -taps.R; k <= taps.R; ++k)
        if (mirror_slice(s + k, S) == s2) b += taps.w[k + taps.R];
    Bm[i] = b;
}

// r_z filter for S <= RZ_REG_S: a thread keeps its pixel's column in
// registers and forms out = B x with the matrix read through the scalar
// cache (every thread of the launch reads the same entries).
constexpr int RZ_REG_S = 32;
__global__ __launch_bounds__(256) void k_rz_filter_reg(float* v0, float* v1, int S, size_t HW,
                                                       const float* __restrict__ Bm, int positive1) {
    // blockIdx.y: 0 filters v0 (amplitude), 1 filters v1 (phase; clipped at 0 with positive1)
    float* const v = blockIdx.y ? v1 : v0;
    const int positive = blockIdx.y ? positive1 : 0;
    const size_t px = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (px >= HW) return;
    float x[RZ_REG_S];
#pragma unroll
    for (int s = 0; s < RZ_REG_S; ++s) x[s] = s < S ? v[(size_t)s * HW + px] : 0.f;
    // a guarded body rather than a break, so that the loop unrolls fully
#pragma unroll
    for (int s = 0; s < RZ_REG_S; ++s) {
        if (s < S) {
            float acc = 0.f;
#pragma unroll
            for (int s2 = 0; s2 < RZ_REG_S; ++s2)
                if (s2 < S) acc = fmaf(Bm[s * S + s2], x[s2], acc);
            v[(size_t)s * HW + px] = positive ? fmaxf(acc, 0.f) : acc;
        }
    }
}

// The same for fields whose slice size is a multiple of 4: a thread owns four
// consecutive pixels (16-byte reads and writes).
__global__ __launch_bounds__(256) void k_rz_filter_reg4(float* v0, float* v1, int S, size_t HW,
                                                        const float* __restrict__ Bm, int positive1) {
    float* const v = blockIdx.y ? v1 : v0;
    const int positive = blockIdx.y ? positive1 : 0;
    const size_t px = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (px >= HW) return;
    float4 x[RZ_REG_S];
#pragma unroll
    for (int s = 0; s < RZ_REG_S; ++s)
        x[s] = s < S ? *reinterpret_cast<const float4*>(v + (size_t)s * HW + px) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int s = 0; s < RZ_REG_S; ++s) {
        if (s < S) {
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int s2 = 0; s2 < RZ_REG_S; ++s2)
                if (s2 < S) {
                    const float b = Bm[s * S + s2];
                    acc.x = fmaf(b, x[s2].x, acc.x);
                    acc.y = fmaf(b, x[s2].y, acc.y);
                    acc.z = fmaf(b, x[s2].z, acc.z);
                    acc.w = fmaf(b, x[s2].w, acc.w);
                }
            if (positive)
                acc = make_float4(fmaxf(acc.x, 0.f), fmaxf(acc.y, 0.f), fmaxf(acc.z, 0.f), fmaxf(acc.w, 0.f));
            *reinterpret_cast<float4*>(v + (size_t)s * HW + px) = acc;
        }
    }
}

// threads per workgroup of the depth filter for S slices (LDS <= 64 KiB)
inline int rz_threads(int S) { return S <= 64 ? 256 : (S <= 128 ? 128 : 64); }

// phase positivity alone (elementwise)
__global__ void k_clip_negative(float* v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        v[i] = fmaxf(v[i], 0.f);
}

// ------------------------------------------------------------ k_z filter
// Mixed-radix (2, 3, 4, 5, 8) Stockham passes through device memory for the
// 3-D transform of the S x H x W object (sides not powers of two, e.g.
// 12 x 640 x 640).  Amplitude and phase travel together as one complex field
// a + i phase: the weight W_a is real and even, so the filtered real and
// imaginary parts are the two filtered fields.

// the element (line l, index i) of an axis sits at off(l) + i * stride with
// off(l) = (l / L1) * P1 + (l % L1) * P0
struct Axis {
    int n;              // transform length
    size_t lines;       // independent lines
    size_t stride;      // element stride along the line
    size_t L1, P1, P0;
    int lines_fast;     // consecutive threads take consecutive lines (else consecutive j)
};

__device__ __forceinline__ float2 cmul_f(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One radix-R pass with Ns = product of the radices before it: thread (l, j),
// j < n / R, reads the R elements j + r n / R, multiplies element r by
// exp(sign 2 pi i r (j mod Ns) / (Ns R)), takes their R-point DFT and writes
// output r to (j / Ns) Ns R + (j mod Ns) + r Ns.
template <int R>
__global__ __launch_bounds__(256) void k_fft_pass(const float2* __restrict__ src, float2* __restrict__ dst, Axis a,
                                                  int Ns, float sign) {
    const int m = a.n / R;
    const size_t total = a.lines * m;
    float2 wr[R];                              // exp(sign 2 pi i q / R)
#pragma unroll
    for (int q = 0; q < R; ++q) {
        float sn, cs;
        sincospif(sign * 2.0f * (float)q / (float)R, &sn, &cs);
        wr[q] = make_float2(cs, sn);
    }
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        size_t l;
        int j;
        if (a.lines_fast) { l = t % a.lines; j = (int)(t / a.lines); }
        else { j = (int)(t % m); l = t / m; }
        const size_t off = (l / a.L1) * a.P1 + (l % a.L1) * a.P0;
        const int k = j % Ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float2 x = src[off + (size_t)(j + r * m) * a.stride];
            float sn, cs;
            sincospif(sign * 2.0f * (float)(r * k) / (float)(Ns * R), &sn, &cs);
            v[r] = cmul_f(x, make_float2(cs, sn));
        }
        float2 o[R];
#pragma unroll
        for (int b = 0; b < R; ++b) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float2 t2 = cmul_f(v[r], wr[(r * b) % R]);
                acc.x += t2.x;
                acc.y += t2.y;
            }
            o[b] = acc;
        }
        const size_t d = (size_t)(j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[off + (d + (size_t)r * Ns) * a.stride] = o[r];
    }
}

__global__ void k_kz_pack(const float* amp, const float* phase, size_t n, float2* z) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        z[i] = make_float2(amp[i], phase[i]);
}
__global__ void k_kz_unpack(const float2* z, size_t n, float* amp, float* phase) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float2 v = z[i];
        amp[i] = v.x;
        phase[i] = v.y;
    }
}

// multiply the 3-D spectrum by W_a(k) / (S H W) (the inverse transform's
// normalisation folded in); k from fftfreq with the pixel size dx and the
// slice spacing dz (1/angstrom), weight evaluated in double
__global__ void k_kz_weight(float2* z, int S, int H, int W, double beta, double alpha, double dx, double dz) {
    const size_t n = (size_t)S * H * W;
    const double norm = 1.0 / (double)n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % W), y = (int)((i / W) % H), s = (int)(i / ((size_t)W * H));
        const double kx = (x < (W + 1) / 2 ? x : x - W) / (W * dx);
        const double ky = (y < (H + 1) / 2 ? y : y - H) / (H * dx);
        const double kz = (s < (S + 1) / 2 ? s : s - S) / (S * dz);
        const double kr2 = kx * kx + ky * ky;
        const double w = (1.0 - (2.0 / 3.14159265358979323846) * atan(beta * beta * kz * kz / (kr2 + 1e-3))) *
                         exp(-alpha * kr2) * norm;
        z[i] = make_float2((float)(z[i].x * w), (float)(z[i].y * w));
    }
}

// radices of n (5s, 3s, then 8s, 4s, 2s); 0 if n has another prime factor
inline int fft_radices(int n, int* rs) {
    int k = 0;
    for (int r : {5, 3})
        while (n % r == 0) { rs[k++] = r; n /= r; }
    while (n % 8 == 0) { rs[k++] = 8; n /= 8; }
    while (n % 4 == 0) { rs[k++] = 4; n /= 4; }
    while (n % 2 == 0) { rs[k++] = 2; n /= 2; }
    return n == 1 ? k : -1;
}

// ------------------------------------------------------------ probe modes
struct cd {
    double re, im;
};
__device__ __forceinline__ cd cd_mul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cd_conj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ cd cd_add(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cd_scale(cd a, double s) { return {a.re * s, a.im * s}; }

// Partial overlaps conj(P_m(r)) P_n(r) summed over one chunk of GRAM_CHUNK
// pixels, in double: one workgroup per (chunk, pair m <= n), written to
// part[pair * nchunk + chunk]; the eigen kernel adds the chunks in order.
__global__ __launch_bounds__(256) void k_probe_gram(const float2* P, int M, int NN, cd* part) {
    const int chunk = blockIdx.x, nchunk = gridDim.x;
    int pair = blockIdx.y, m = 0;
    const int pair_id = pair;
    while (pair >= M - m) { pair -= M - m; ++m; }
    const int n = m + pair;
    const float2* a = P + (size_t)m * NN;
    const float2* b = P + (size_t)n * NN;
    double re = 0.0, im = 0.0;
    const int r1 = min(NN, (chunk + 1) * GRAM_CHUNK);
    for (int r = chunk * GRAM_CHUNK + threadIdx.x; r < r1; r += blockDim.x) {
        const float2 x = a[r], y = b[r];
        re += (double)x.x * y.x + (double)x.y * y.y;       // conj(x) y
        im += (double)x.x * y.y - (double)x.y * y.x;
    }
    __shared__ double sr[256], si[256];
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)pair_id * nchunk + chunk] = {sr[0], si[0]};
}

// Eigenvectors of the Hermitian overlap matrix (summed from the chunk
// partials) by cyclic complex Jacobi
// rotations in double (one workgroup, thread k owning row / column k), then
// ordered by decreasing eigenvalue; each eigenvector is scaled by a unit
// phase so that its largest-magnitude entry (first of equals) is real and
// positive.  Writes V (M x M, column k = mode k's mixing coefficients) as
// float pairs and the eigenvalues.
__global__ __launch_bounds__(64) void k_probe_eig(const cd* part, int nchunk, int M, float2* Vout, double* lam_out) {
    __shared__ cd A[ORTH_MAX_M * ORTH_MAX_M], V[ORTH_MAX_M * ORTH_MAX_M];
    __shared__ double lam[ORTH_MAX_M];
    __shared__ int order[ORTH_MAX_M];
    __shared__ double off;
    const int k = threadIdx.x;
    for (int i = k; i < M * M; i += blockDim.x) V[i] = {(i / M) == (i % M) ? 1.0 : 0.0, 0.0};
    // overlap matrix from the chunk sums (fixed order)
    for (int pid = k; pid < M * (M + 1) / 2; pid += blockDim.x) {
        int pr = pid, m = 0;
        while (pr >= M - m) { pr -= M - m; ++m; }
        const int n = m + pr;
        double re = 0.0, im = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) {
            re += part[(size_t)pid * nchunk + ch].re;
            im += part[(size_t)pid * nchunk + ch].im;
        }
        A[m * M + n] = {re, m == n ? 0.0 : im};
        A[n * M + m] = {re, m == n ? 0.0 : -im};
    }
    __syncthreads();
    double scale = 0.0;
    for (int i = 0; i < M; ++i) scale += A[i * M + i].re;
    const double tol = 1e-28 * scale * scale;     // off-diagonal norm 1e-14 of the trace
    for (int sweep = 0; sweep < 64; ++sweep) {
        if (k == 0) {
            double s = 0.0;
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j)
                    if (i != j) s += A[i * M + j].re * A[i * M + j].re + A[i * M + j].im * A[i * M + j].im;
            off = s;
        }
        __syncthreads();
        if (off <= tol) break;
        for (int p = 0; p < M - 1; ++p)
            for (int q = p + 1; q < M; ++q) {
                const cd apq = A[p * M + q];
                const double mag = sqrt(apq.re * apq.re + apq.im * apq.im);
                if (mag == 0.0) continue;                       // uniform: every thread reads the same value
                // U = D P: D_qq = exp(-i alpha) makes the (p, q) entry real
                // (alpha = arg a_pq), P the real Jacobi rotation that zeroes it
                const cd e = {apq.re / mag, -apq.im / mag};     // exp(-i alpha)
                const double zeta = (A[q * M + q].re - A[p * M + p].re) / (2.0 * mag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(zeta * zeta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                __syncthreads();
                // columns p, q of A U and of V U (thread k: row k)
                if (k < M) {
                    const cd akp = A[k * M + p], akq = cd_mul(A[k * M + q], e);
                    A[k * M + p] = {c * akp.re - s * akq.re, c * akp.im - s * akq.im};
                    A[k * M + q] = {s * akp.re + c * akq.re, s * akp.im + c * akq.im};
                    const cd vkp = V[k * M + p], vkq = cd_mul(V[k * M + q], e);
                    V[k * M + p] = {c * vkp.re - s * vkq.re, c * vkp.im - s * vkq.im};
                    V[k * M + q] = {s * vkp.re + c * vkq.re, s * vkp.im + c * vkq.im};
                }
                __syncthreads();
                // rows p, q of U^H (A U) (thread k: column k)
                if (k < M) {
                    const cd bpk = A[p * M + k], bqk = cd_mul(A[q * M + k], cd_conj(e));
                    A[p * M + k] = {c * bpk.re - s * bqk.re, c * bpk.im - s * bqk.im};
                    A[q * M + k] = {s * bpk.re + c * bqk.re, s * bpk.im + c * bqk.im};
                }
                __syncthreads();
                if (k == 0) {
                    A[p * M + q] = {0.0, 0.0};
                    A[q * M + p] = {0.0, 0.0};
                    A[p * M + p].im = 0.0;
                    A[q * M + q].im = 0.0;
                }
                __syncthreads();
            }
    }
    if (k == 0) {
        for (int i = 0; i < M; ++i) {
            lam[i] = A[i * M + i].re;
            order[i] = i;
        }
        for (int i = 0; i < M; ++i)                       // selection sort, decreasing; stable for ties
            for (int j = i + 1; j < M; ++j)
                if (lam[order[j]] > lam[order[i]]) {
                    const int tmp = order[i];
                    order[i] = order[j];
                    order[j] = tmp;
                }
    }
    __syncthreads();
    if (k < M) {                                          // thread k: output column k
        const int src = order[k];
        int best = 0;
        double bm = -1.0;
        for (int m = 0; m < M; ++m) {
            const cd x = V[m * M + src];
            const double a = x.re * x.re + x.im * x.im;
            if (a > bm) { bm = a; best = m; }
        }
        const cd x = V[best * M + src];
        const double r = sqrt(x.re * x.re + x.im * x.im);
        const cd ph = r > 0 ? cd{x.re / r, -x.im / r} : cd{1.0, 0.0};
        for (int m = 0; m < M; ++m) {
            const cd y = cd_mul(V[m * M + src], ph);
            Vout[m * M + k] = make_float2((float)y.re, (float)y.im);
        }
        lam_out[k] = lam[src];
    }
}

// Q_k(r) = sum_m V[m][k] P_m(r), in place: a workgroup stages the M values of
// its 256 pixels in LDS before writing.  Dynamic LDS: M * 256 float2 + M^2 float2.
__global__ __launch_bounds__(256) void k_probe_mix(float2* P, int M, int NN, const float2* V) {
    extern __shared__ float2 sm[];
    float2* vals = sm;                        // vals[m * 256 + t]
    float2* Vs = sm + (size_t)M * 256;
    const int t = threadIdx.x;
    const int r = blockIdx.x * 256 + t;
    for (int i = t; i < M * M; i += 256) Vs[i] = V[i];
    for (int m = 0; m < M; ++m) vals[m * 256 + t] = r < NN ? P[(size_t)m * NN + r] : make_float2(0.f, 0.f);
    __syncthreads();
    if (r >= NN) return;
    for (int kk = 0; kk < M; ++kk) {
        float re = 0.f, im = 0.f;
        for (int m = 0; m < M; ++m) {
            const float2 v = Vs[m * M + kk], p = vals[m * 256 + t];
            re = fmaf(v.x, p.x, fmaf(-v.y, p.y, re));
            im = fmaf(v.x, p.y, fmaf(v.y, p.x, im));
        }
        P[(size_t)kk * NN + r] = make_float2(re, im);
    }
}

}  // namespace ptyr
