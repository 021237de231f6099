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
// The 3-D transform of one S x H x W object stack (sides with no prime factor
// other than 2, 3 and 5, e.g. 12 x 640 x 640) runs as line passes, each one
// round trip through device memory: a workgroup loads a tile of lines into
// LDS, runs every radix stage of their DFTs there (Stockham stages in place,
// each butterfly's values held in registers across a barrier) and writes the
// tile back.  Amplitude and phase travel as one complex field a + i phase:
// the weight W_a is real and even in k, so the filtered real and imaginary
// parts are the two filtered fields.  Per call: forward x (reading amplitude
// and phase), forward y, one z pass (forward, weight, inverse), inverse y,
// inverse x (writing amplitude and phase): five passes, 16 bytes per voxel
// each.

constexpr int KZ_THREADS = 1024;
constexpr int KZ_LDS = 8192;        // complex values of LDS per workgroup (64 KiB): tile + twiddles
constexpr int KZ_EPT = KZ_LDS / KZ_THREADS;
constexpr int KZ_MAX_SIDE = KZ_LDS / 2;
constexpr int KZ_MAX_RAD = 16;
constexpr int KZ_BATCH = 8;        // loads in flight per thread

enum : int { KZ_IN_FIELDS = 1, KZ_OUT_FIELDS = 2, KZ_FILTER = 4 };

// One axis: the lines form `groups` groups of lpg lines; line c of group q
// starts at q * gs + c * gc and its element i sits i * gi further.  A tile is
// nl consecutive lines of one group (the last tile of a group may hold fewer);
// tile t covers group t / tpg.
struct KzPass {
    int n, lg, ls, lpg, tpg;    // line length, log2 lines per tile, LDS row pitch (rows), lines per group, tiles per group
    int tiles;                  // tiles of the pass (the grid is rounded up to a multiple of 8)
    size_t gs, gc, gi;
    int nrad;
    unsigned long long rads;    // radix k in bits 4k .. 4k + 3
    const float2* tw;           // exp(-2 pi i k / n), k < n
};
struct KzWeight {
    int S, H, W;
    double beta, alpha, dx, dz;
};

__device__ __forceinline__ float2 kz_mul_i(float2 a, int sg) {       // a * (sg i)
    return sg > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// R-point DFT X_b = sum_q x_q exp(SG 2 pi i q b / R) in place
template <int R, int SG> __device__ __forceinline__ void kz_dft(float2* x) {
    if constexpr (R == 2) {
        const float2 a = x[0], b = x[1];
        x[0] = make_float2(a.x + b.x, a.y + b.y);
        x[1] = make_float2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const float2 y0 = make_float2(x[0].x + x[2].x, x[0].y + x[2].y);
        const float2 y1 = make_float2(x[0].x - x[2].x, x[0].y - x[2].y);
        const float2 y2 = make_float2(x[1].x + x[3].x, x[1].y + x[3].y);
        const float2 y3 = kz_mul_i(make_float2(x[1].x - x[3].x, x[1].y - x[3].y), SG);
        x[0] = make_float2(y0.x + y2.x, y0.y + y2.y);
        x[2] = make_float2(y0.x - y2.x, y0.y - y2.y);
        x[1] = make_float2(y1.x + y3.x, y1.y + y3.y);
        x[3] = make_float2(y1.x - y3.x, y1.y - y3.y);
    } else if constexpr (R == 8) {
        float2 e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
        kz_dft<4, SG>(e);
        kz_dft<4, SG>(o);
        // exp(SG 2 pi i k / 8) for k = 1, 2, 3
        constexpr float r = 0.70710678118654752440f;
        o[1] = make_float2(r * (o[1].x - SG * o[1].y), r * (o[1].y + SG * o[1].x));
        o[2] = kz_mul_i(o[2], SG);
        o[3] = make_float2(r * (-o[3].x - SG * o[3].y), r * (-o[3].y + SG * o[3].x));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = make_float2(e[k].x + o[k].x, e[k].y + o[k].y);
            x[k + 4] = make_float2(e[k].x - o[k].x, e[k].y - o[k].y);
        }
    } else if constexpr (R == 3) {
        constexpr float h = 0.86602540378443864676f;          // sin(2 pi / 3)
        const float2 s = make_float2(x[1].x + x[2].x, x[1].y + x[2].y);
        const float2 t = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
        const float2 u = kz_mul_i(make_float2(h * (x[1].x - x[2].x), h * (x[1].y - x[2].y)), SG);
        x[0] = make_float2(x[0].x + s.x, x[0].y + s.y);
        x[1] = make_float2(t.x + u.x, t.y + u.y);
        x[2] = make_float2(t.x - u.x, t.y - u.y);
    } else {
        static_assert(R == 5, "radix 2, 3, 4, 5 or 8");
        constexpr float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;   // cos(2 pi / 5), cos(4 pi / 5)
        constexpr float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;    // sin(2 pi / 5), sin(4 pi / 5)
        const float2 t1 = make_float2(x[1].x + x[4].x, x[1].y + x[4].y);
        const float2 t2 = make_float2(x[2].x + x[3].x, x[2].y + x[3].y);
        const float2 d1 = make_float2(x[1].x - x[4].x, x[1].y - x[4].y);
        const float2 d2 = make_float2(x[2].x - x[3].x, x[2].y - x[3].y);
        const float2 a1 = make_float2(x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y);
        const float2 a2 = make_float2(x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y);
        const float2 b1 = kz_mul_i(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y), SG);
        const float2 b2 = kz_mul_i(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y), SG);
        x[0] = make_float2(x[0].x + t1.x + t2.x, x[0].y + t1.y + t2.y);
        x[1] = make_float2(a1.x + b1.x, a1.y + b1.y);
        x[4] = make_float2(a1.x - b1.x, a1.y - b1.y);
        x[2] = make_float2(a2.x + b2.x, a2.y + b2.y);
        x[3] = make_float2(a2.x - b2.x, a2.y - b2.y);
    }
}

// j / d for 0 <= j < 2^13 and 1 <= d < 2^13 from a float reciprocal: the
// product (j + 1/2) (1/d) is within 2^-23 (j + 1/2) / d of the exact quotient,
// less than its distance 1 / (2 d) to the nearest integer
__device__ __forceinline__ int kz_div(int j, float inv_d) { return (int)(((float)j + 0.5f) * inv_d); }

// One Stockham stage over the tile's lines of length n in LDS (element i of
// line c at c * ls + i * es; lines c >= cnt of a short tile are skipped),
// Ns = product of the earlier radices: butterfly (c, j), j < n / R, takes
// elements j + r n / R, multiplies element r by exp(SG 2 pi i r (j mod Ns) /
// (Ns R)), takes their R-point DFT and puts output r at (j / Ns) Ns R +
// (j mod Ns) + r Ns.  tw[k] = exp(-2 pi i k / n).  Butterfly b of the tile is
// (c, j) = (b mod nl, b / nl) (nl = 2^lg lines per tile).  Every thread reads
// all its butterflies before the barrier and writes them after it, so the
// stage runs in place.
template <int R, int SG>
__device__ void kz_stage(float2* z, const float2* tw, int n, int lg, int cnt, int ls, int es, int Ns) {
    constexpr int Q = (KZ_EPT + R - 1) / R;
    const int nl = 1 << lg, m = n / R, total = m << lg, tstep = n / (Ns * R);
    const float inv_ns = 1.0f / (float)Ns;
    float2 v[Q][R];
    int out[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = (int)threadIdx.x + q * KZ_THREADS;
        const int c = b & (nl - 1), j = b >> lg;
        out[q] = -1;
        if (b < total && c < cnt) {
            const int jd = kz_div(j, inv_ns), k = j - jd * Ns;
            const int base = c * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float2 x = z[base + (j + r * m) * es];
                if (r == 0) {
                    v[q][0] = x;
                } else {
                    const float2 w = tw[r * k * tstep];
                    const float wy = SG < 0 ? w.y : -w.y;
                    v[q][r] = make_float2(x.x * w.x - x.y * wy, x.x * wy + x.y * w.x);
                }
            }
            kz_dft<R, SG>(v[q]);
            out[q] = base + (jd * Ns * R + k) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (out[q] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) z[out[q] + r * Ns * es] = v[q][r];
        }
    __syncthreads();
}

template <int SG>
__device__ void kz_line_dft(float2* z, const float2* tw, const KzPass& a, int cnt, int ls, int es) {
    int Ns = 1;
    for (int p = 0; p < a.nrad; ++p) {
        const int R = (int)((a.rads >> (4 * p)) & 15);
        switch (R) {
            case 2: kz_stage<2, SG>(z, tw, a.n, a.lg, cnt, ls, es, Ns); break;
            case 3: kz_stage<3, SG>(z, tw, a.n, a.lg, cnt, ls, es, Ns); break;
            case 4: kz_stage<4, SG>(z, tw, a.n, a.lg, cnt, ls, es, Ns); break;
            case 5: kz_stage<5, SG>(z, tw, a.n, a.lg, cnt, ls, es, Ns); break;
            default: kz_stage<8, SG>(z, tw, a.n, a.lg, cnt, ls, es, Ns); break;
        }
        Ns *= R;
    }
}

// One line pass.  F: KZ_IN_FIELDS reads amplitude and phase instead of z,
// KZ_OUT_FIELDS writes them instead of z, KZ_FILTER runs the forward
// transform, the weight and the inverse transform (the z pass: its lines are
// the H W pixels, line p at spectral (y, x) = (p / W, p mod W)); otherwise one
// transform of sign SG.  Rows (x: lines contiguous in memory) sit in LDS as
// [c][i] with row pitch a.ls; columns (y, z) as [i][c] with pitch nl.
// Dynamic LDS: kz_lds_bytes(a).
template <int F, int SG>
__global__ __launch_bounds__(KZ_THREADS) void k_kz_lines(float2* z, float* amp, float* phase, KzPass a, KzWeight w) {
    extern __shared__ float2 kz_lds[];
    // workgroups are dealt to the 8 XCDs in turn; tile t runs as workgroup
    // (t mod G8) * 8 + t / G8, so neighbouring tiles (which share cache lines
    // along a row in the column passes) run side by side on one XCD's L2
    const int g8 = (int)gridDim.x >> 3, tt = ((int)blockIdx.x & 7) * g8 + ((int)blockIdx.x >> 3);
    if (tt >= a.tiles) return;
    const int q = tt / a.tpg, u = tt % a.tpg;
    const int nl = 1 << a.lg, c0 = u * nl, cnt = min(nl, a.lpg - c0);
    const int n = a.n;
    const bool rows = a.gi == 1;
    const int ls = rows ? a.ls : 1, es = rows ? 1 : nl;
    float2* t = kz_lds;
    float2* tw = kz_lds + (size_t)nl * (rows ? a.ls : n);
    for (int k = threadIdx.x; k < n; k += KZ_THREADS) tw[k] = a.tw[k];
    const size_t base = (size_t)q * a.gs + (size_t)c0 * a.gc;
    // tile element e: rows e = c n + i (contiguous in memory), columns
    // e = i nl + c; returns the LDS slot, or -1 past the tile
    const float inv_n = 1.0f / (float)n;
    auto slot = [&](int e, size_t& g) -> int {
        if (rows) {
            if (e >= cnt * n) return -1;
            const int c = kz_div(e, inv_n), i = e - c * n;
            g = base + (size_t)e;
            return c * ls + i;
        }
        const int c = e & (nl - 1), i = e >> a.lg;
        if (i >= n || c >= cnt) return -1;
        g = base + (size_t)c + (size_t)i * a.gi;
        return e;
    };
    // loads in batches of KZ_BATCH per thread, all in flight before the
    // batch is put into LDS
    const int ne = rows ? cnt * n : n << a.lg;
    for (int e0 = 0; e0 < ne; e0 += KZ_BATCH * KZ_THREADS) {
        float2 v[KZ_BATCH];
        int sl[KZ_BATCH];
#pragma unroll
        for (int r = 0; r < KZ_BATCH; ++r) {
            size_t g = 0;
            sl[r] = slot(e0 + (int)threadIdx.x + r * KZ_THREADS, g);
            if (sl[r] >= 0) {
                if constexpr ((F & KZ_IN_FIELDS) != 0) v[r] = make_float2(amp[g], phase[g]);
                else v[r] = z[g];
            }
        }
#pragma unroll
        for (int r = 0; r < KZ_BATCH; ++r)
            if (sl[r] >= 0) t[sl[r]] = v[r];
    }
    __syncthreads();
    if constexpr ((F & KZ_FILTER) != 0) {
        kz_line_dft<-1>(t, tw, a, cnt, ls, es);
        // W_a(k) / (S H W): per pixel A = beta^2 / (k_r^2 + 1e-3) and
        // E = exp(-alpha k_r^2) / (S H W) (k_r^2 in double), per element
        // (1 - (2 / pi) atan(A k_z^2)) E; k from fftfreq with the pixel size
        // dx and the slice spacing dz (1/angstrom).  nl divides KZ_THREADS,
        // so every element a thread visits belongs to its pixel c.
        const int c = (int)threadIdx.x & (nl - 1);
        float fa = 0.f, fe = 0.f;
        if (c < cnt) {
            const int p = c0 + c, y = p / w.W, x = p - y * w.W;
            const double kx = (x < (w.W + 1) / 2 ? x : x - w.W) / (w.W * w.dx);
            const double ky = (y < (w.H + 1) / 2 ? y : y - w.H) / (w.H * w.dx);
            const double kr2 = kx * kx + ky * ky;
            fa = (float)(w.beta * w.beta / (kr2 + 1e-3));
            fe = (float)(exp(-w.alpha * kr2) / ((double)w.S * w.H * w.W));
        }
        for (int e = threadIdx.x; e < (n << a.lg); e += KZ_THREADS) {
            const int s = e >> a.lg;
            if (c < cnt) {
                const float kz = (float)((s < (w.S + 1) / 2 ? s : s - w.S) / (w.S * w.dz));
                const float wt = (1.0f - 0.63661977236758134308f * atanf(fa * kz * kz)) * fe;
                float2& v = t[c * ls + s * es];
                v = make_float2(v.x * wt, v.y * wt);
            }
        }
        __syncthreads();
        kz_line_dft<+1>(t, tw, a, cnt, ls, es);
    } else {
        kz_line_dft<SG>(t, tw, a, cnt, ls, es);
    }
    for (int e = threadIdx.x; e < ne; e += KZ_THREADS) {
        size_t g = 0;
        const int sl = slot(e, g);
        if (sl < 0) continue;
        const float2 x = t[sl];
        if constexpr ((F & KZ_OUT_FIELDS) != 0) {
            amp[g] = x.x;
            phase[g] = x.y;
        } else {
            z[g] = x;
        }
    }
}

// exp(-2 pi i k / n) for k < n (in double, rounded to float)
__global__ void k_kz_twiddles(float2* tw, int n) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(2.0 * k / n, &sn, &cs);
        tw[k] = make_float2((float)cs, (float)-sn);
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

// the line pass over `groups` groups of lpg lines of length n with the radices
// rad[0..nrad): 2^lg lines per tile, the most up to nl_max (at most
// KZ_THREADS) whose tile and twiddle table fit in KZ_LDS; rows
// (gi == 1) get a row pitch of n + 8 where it fits (LDS reads of the lines'
// elements side by side then fall in different banks); *grid = the tiles
inline KzPass kz_pass(int n, int groups, int lpg, size_t gs, size_t gc, size_t gi, const int* rad, int nrad,
                      int nl_max, const float2* tw, int* grid) {
    KzPass a{};
    a.tw = tw;
    a.n = n;
    a.lpg = lpg;
    a.gs = gs;
    a.gc = gc;
    a.gi = gi;
    a.nrad = nrad;
    for (int k = 0; k < nrad && k < KZ_MAX_RAD; ++k) a.rads |= (unsigned long long)rad[k] << (4 * k);
    const bool rows = gi == 1;
    auto fits = [&](int nl, int pitch) { return nl * pitch + n <= KZ_LDS; };
    a.ls = rows && fits(1, n + 8) ? n + 8 : n;
    a.lg = 0;
    while ((2 << a.lg) <= nl_max && fits(2 << a.lg, a.ls)) ++a.lg;
    a.tpg = (lpg + (1 << a.lg) - 1) >> a.lg;
    a.tiles = groups * a.tpg;
    *grid = (a.tiles + 7) & ~7;
    return a;
}
// tile and twiddles
inline size_t kz_lds_bytes(const KzPass& a) {
    const size_t nl = (size_t)1 << a.lg;
    return (nl * (a.gi == 1 ? a.ls : a.n) + a.n) * sizeof(float2);
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
