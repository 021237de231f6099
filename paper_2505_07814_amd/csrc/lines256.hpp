// lines256.hpp - the multislice forward model and its gradient for N = 256.
//
// A 256 x 256 complex64 wave (512 KiB) does not fit one compute unit, so it
// stays in device memory (L2 / Infinity Cache resident for the batch) and
// each slice is two line passes over all (row, mode) chains of the batch:
//
//   row pass    : inverse DFT along x (phi_s), transmit by O_s, DFT along x
//   column pass : DFT along y (full 2-D spectrum), multiply by H, inverse DFT
//                 along y
//
// The wave between a column pass and the next row pass, Z_s (y, k_x), is the
// one wave kept per slice: the column pass writes it into slice s's slot of
// the store and the row pass reads it from there.  The gradient rebuilds from
// it both phi_s (the row pass's inverse along x, bitwise the forward's) and
// the spectrum Y_s (a DFT along y), so the forward moves four waves per slice
// instead of six (no separate phi_s and Y_s stores) at the price of one line
// DFT more in each gradient pass.
//
// A workgroup transforms 16 lines of 256 points with the register / LDS line
// machinery of wave.hpp (16 lanes per line, 16 values per lane).  Row passes
// map lanes along x and column passes map lanes across the 16 columns, so
// both read and write 128-byte contiguous segments.  The gradient runs the
// same two passes per slice in reverse with the adjoint operations.
#pragma once
#include "kernels.hpp"

namespace ptyr {

constexpr int N256 = 256;
constexpr int LINES256 = 16;                   // lines per workgroup
constexpr int NBLK256 = N256 / LINES256;       // line blocks per wave

// lanes along the line (row passes): thread = line * 16 + lane
struct RowGeo256 {
    static constexpr int NL = 256, L = 16, SB = 17, SL = 272;
    static constexpr bool WAVE_LOCAL = true;        // the 16 lanes of a line are in one wave
};
// lanes across lines (column passes): thread = lane * 16 + line, so the lanes
// of a line span all four waves and an exchange needs a workgroup barrier
struct ColGeo256 {
    static constexpr int NL = 256, L = 16, SB = 17, SL = 274;
    static constexpr bool WAVE_LOCAL = false;
};
constexpr int LDS256 = (LINES256 - 1) * 274 + 15 * 17 + 16;

struct Tables256 {
    float4 tw[N256];       // tw[b*16 + c] = exp(-2 pi i c b / 256)
    float4 h[N256];        // propagator factor along the pass direction
    float2 r[N256];        // shift ramp along the pass direction
    float4 hl[LINES256];   // propagator factor of each line of the block (column passes)
    float2 rl[LINES256];   // shift ramp of each line of the block (column passes)
};

// The factors of one batch position, both axes (0: y, 1: x), all 256
// frequencies: propagator h[axis][k] = exp(-i pi lam dz k^2 + 2 pi i dz k
// tan th_axis) and shift ramp r[axis][k] = exp(-2 pi i q dr_axis), as
// compensated unit pairs (the ramp's low parts are not used).  Computed once
// per forward or gradient call by k256_tables instead of in every workgroup
// of every pass.
struct PosTab256 {
    float4 h[2][N256];
    float2 r[2][N256];
};

// twiddles (block 0) and the factors of batch position blockIdx.x; 256
// threads, one per frequency
__global__ __launch_bounds__(256) void k256_tables(WaveArgs a, float4* tw, PosTab256* tab) {
    const double pi_d = 3.14159265358979323846;
    const int n = threadIdx.x, j = blockIdx.x;
    double s, c;
    if (j == 0) {
        sincos(-2.0 * pi_d * (double)((n / 16) * (n % 16)) / N256, &s, &c);
        tw[n] = unit_pair(c, s);
    }
    const PosInfo pi = a.pinfo[j];
    if (pi.ty < 0) return;                           // the passes skip the row
    const float* th = a.global_tilt ? a.tilt : a.tilt + 2 * pi.row;
    const double dz = *a.dz;
    const double q = (double)sfreq<N256>(n) / N256, k = q / a.dx;
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const double tan_a = tan((double)th[ax]), dr = ax == 0 ? pi.dry : pi.drx;
        sincos(-pi_d * a.lam * dz * k * k + 2.0 * pi_d * dz * k * tan_a, &s, &c);
        tab[j].h[ax][n] = unit_pair(c, s);
        sincos(-2.0 * pi_d * q * dr, &s, &c);
        const float4 r = unit_pair(c, s);
        tab[j].r[ax][n] = make_float2(r.x, r.y);
    }
}

// A workgroup's tables: the twiddles and, for its position, the factors along
// the pass direction (AXIS 0: y, 1: x) for all 256 frequencies and those of
// the block's 16 lines along the other axis.
template <int AXIS>
__device__ __forceinline__ void load256(Tables256& t, const float4* tw, const PosTab256* tab, int j, int line0) {
    const int n = threadIdx.x;                       // blockDim.x == 256
    const PosTab256& T = tab[j];
    t.tw[n] = tw[n];
    t.h[n] = T.h[AXIS][n];
    t.r[n] = T.r[AXIS][n];
    if (n < LINES256) {
        t.hl[n] = T.h[1 - AXIS][line0 + n];
        t.rl[n] = T.r[1 - AXIS][line0 + n];
    }
    __syncthreads();
}

// block of 16 rows (row passes) or 16 columns (column passes) of one wave:
// register r of lane c of line l is element (line0 + l, c + 16 r) for rows and
// (c + 16 r, line0 + l) for columns.
__device__ __forceinline__ void rows_load(float2 (&v)[16], const float2* w, int y, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = w[y * N256 + c + 16 * r];
}
__device__ __forceinline__ void rows_store(const float2 (&v)[16], float2* w, int y, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) w[y * N256 + c + 16 * r] = v[r];
}
__device__ __forceinline__ void cols_load(float2 (&v)[16], const float2* w, int x, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = w[(c + 16 * r) * N256 + x];
}
__device__ __forceinline__ void cols_store(const float2 (&v)[16], float2* w, int x, int c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) w[(c + 16 * r) * N256 + x] = v[r];
}

// Kept waves (phi_s, Y_s, far field) are written and read by passes of the
// same geometry, register-major per line block: register r of thread t of
// block blk at blk 4096 + r 256 + t, so each access instruction moves one
// contiguous 512-byte run per wave.
__device__ __forceinline__ void keep_store(const float2 (&v)[16], float2* w, int blk) {
#pragma unroll
    for (int r = 0; r < 16; ++r) (w + blk * (LINES256 * N256) + r * 256)[threadIdx.x] = v[r];
}
__device__ __forceinline__ void keep_load(float2 (&v)[16], const float2* w, int blk) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = (w + blk * (LINES256 * N256) + r * 256)[threadIdx.x];
}

struct Pass256 {
    WaveArgs a;
    float2* wave;          // B x M x 256 x 256 working waves
    const float4* tw;      // twiddles (k256_tables)
    const PosTab256* tab;  // per batch position factors (k256_tables)
    int s;                 // slice of the pass
    int mg;                // gradient row pass: probe modes per workgroup (divides the probe modes)
};

// Forward row pass of slice s: wave holds (y, k_x) of the previous column
// pass (for s == 0 the shifted probe still lacking its x ramp); keeps phi_s,
// transmits by O_s and transforms along x.
__global__ __launch_bounds__(256) void k256_fwd_row(Pass256 P) {
    __shared__ float2 lds[LDS256];
    __shared__ Tables256 tab;
    const WaveArgs& a = P.a;
    const int ch = a.chain0 + blockIdx.x / NBLK256, blk = blockIdx.x % NBLK256;
    const int j = ch / a.M;
    const PosInfo pi = a.pinfo[j];
    if (pi.ty < 0) return;
    const int l = threadIdx.x / 16, c = threadIdx.x % 16, y = blk * LINES256 + l;
    load256<1>(tab, P.tw, P.tab, j, blk * LINES256);
    float2* w = P.wave + (size_t)ch * N256 * N256;
    const Slots<N256> sl(a, ch);
    const bool full = sl.base && a.keep == KEEP_FULL;
    float2 v[16], ov[16];
    rows_load(v, full ? sl.phi(P.s) : w, y, c);
    // the object patch is read now, so that its latency overlaps the line DFT
    // (three workgroups per CU by LDS leave room for the extra registers)
    const float2* Os = chain_object(a, ch % a.M) + (size_t)P.s * a.H * a.W + (size_t)(pi.ty + y) * a.W + pi.tx;
#pragma unroll
    for (int r = 0; r < 16; ++r) ov[r] = Os[c + 16 * r];
    if (P.s == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = cmul(v[r], tab.r[c + 16 * r]);
    }
    mid2nat<RowGeo256, +1>(v, lds, tab.tw, l, c);                      // phi_s (space)
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cmul(v[r], ov[r]);
    nat2mid<RowGeo256, -1>(v, lds, tab.tw, l, c);
    rows_store(v, w, y, c);
}

// Forward column pass: s < 0 builds the shifted probe (inverse along y of
// Phat R_y / N); 0 <= s < S-1 propagates to slice s+1 (keeping Y'_{s+1});
// s == S-1 forms the far field and its intensity.
__global__ __launch_bounds__(256) void k256_fwd_col(Pass256 P) {
    __shared__ float2 lds[LDS256];
    __shared__ Tables256 tab;
    const WaveArgs& a = P.a;
    const int ch = a.chain0 + blockIdx.x / NBLK256, blk = blockIdx.x % NBLK256;
    const int j = ch / a.M, m = ch % a.M;
    const PosInfo pi = a.pinfo[j];
    const int l = threadIdx.x % 16, c = threadIdx.x / 16, x = blk * LINES256 + l;
    float* Iout = a.Imode + (size_t)ch * N256 * N256;
    if (pi.ty < 0) {
        if (P.s == a.S - 1) {
#pragma unroll
            for (int r = 0; r < 16; ++r) Iout[(c + 16 * r) * N256 + x] = 0.f;
        }
        return;
    }
    load256<0>(tab, P.tw, P.tab, j, blk * LINES256);
    float2* w = P.wave + (size_t)ch * N256 * N256;
    const Slots<N256> sl(a, ch);
    const bool full = sl.base && a.keep == KEEP_FULL;
    float2 v[16];
    if (P.s < 0) {
        cols_load(v, chain_probe(a, m, N256 * N256), x, c);
        const float sc = 1.0f / N256;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = cscale(cmul(v[r], tab.r[c + 16 * r]), sc);
        mid2nat<ColGeo256, +1>(v, lds, tab.tw, l, c);
        cols_store(v, full ? sl.phi(0) : w, x, c);                      // Z_0
        return;
    }
    cols_load(v, w, x, c);
    nat2mid<ColGeo256, -1>(v, lds, tab.tw, l, c);                       // full 2-D spectrum (raw)
    if (P.s < a.S - 1) {
        const float4 hx = tab.hl[l];
        const float sc = 1.0f / ((float)N256 * N256);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = cscale(tmul<false>(tmul<false>(v[r], tab.h[c + 16 * r]), hx), sc);
        mid2nat<ColGeo256, +1>(v, lds, tab.tw, l, c);
        cols_store(v, full ? sl.phi(P.s + 1) : w, x, c);                 // Z_{s+1}
    } else {
        if (full) keep_store(v, sl.far(), blk);
        const float s2 = 1.0f / ((float)N256 * N256);
#pragma unroll
        for (int r = 0; r < 16; ++r) Iout[(c + 16 * r) * N256 + x] = cabs2(v[r]) * s2;
    }
}

// Gradient column pass.  s == S: start, G_Psi = w F[chi_{S-1}] -> inverse
// along y.  1 <= s < S: the adjoint of slice s's propagation (after the row
// pass of slice s): G^ -> dz / tilt partial sums with Y'_s -> conj(H) G^ / N^2
// -> inverse along y.  s == 0: probe-spectrum and position terms.
__global__ __launch_bounds__(256) void k256_grad_col(Pass256 P) {
    __shared__ float2 lds[LDS256];
    __shared__ Tables256 tab;
    const WaveArgs& a = P.a;
    const int ch = a.chain0 + blockIdx.x / NBLK256, blk = blockIdx.x % NBLK256;
    const int j = ch / a.M, m = ch % a.M;
    const PosInfo pi = a.pinfo[j];
    const int l = threadIdx.x % 16, c = threadIdx.x / 16, x = blk * LINES256 + l;
    double* part = a.part + ((size_t)ch * NBLK256 + blk) * 8;
    if (pi.ty < 0) {
        if (P.s == 0) {
            float2* gP = a.gPhat + (size_t)ch * N256 * N256;
#pragma unroll
            for (int r = 0; r < 16; ++r) gP[(c + 16 * r) * N256 + x] = make_float2(0.f, 0.f);
            if (threadIdx.x < 8) part[threadIdx.x] = 0.0;
        }
        return;
    }
    load256<0>(tab, P.tw, P.tab, j, blk * LINES256);
    const Slots<N256> sl(a, ch);
    float2* w = P.wave + (size_t)ch * N256 * N256;
    const float inv_n = 1.0f / N256, inv_n2 = 1.0f / ((float)N256 * N256);
    float2 v[16];
    if (P.s == a.S) {
        keep_load(v, sl.far(), blk);
        const float* wj = a.wgt + (size_t)j * N256 * N256;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = cscale(v[r], wj[(c + 16 * r) * N256 + x] * inv_n2);
        mid2nat<ColGeo256, +1>(v, lds, tab.tw, l, c);
        cols_store(v, w, x, c);
        if (threadIdx.x < 8) part[threadIdx.x] = 0.0;
        return;
    }
    cols_load(v, w, x, c);
    float2 yv_[16];                      // Z_s, read now so that its latency overlaps the DFT
    if (P.s > 0) cols_load(yv_, sl.phi(P.s), x, c);
    nat2mid<ColGeo256, -1>(v, lds, tab.tw, l, c);                       // G^ (raw), (k_y, k_x)
    if (P.s > 0) {
        // Y'_s = F_y[Z_s] / N: the forward's inverse along y undone (1/N is exact)
        nat2mid<ColGeo256, -1>(yv_, lds, tab.tw, l, c);
#pragma unroll
        for (int r = 0; r < 16; ++r) yv_[r] = cscale(yv_[r], inv_n);
    }
    // partial sums in double (see k_gradient)
    const double dk = 1.0 / (N256 * a.dx);
    const double kx = sfreq<N256>(x) * dk, kx2 = kx * kx;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (P.s > 0) {
        const float4 hx = tab.hl[l];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ky_i = c + 16 * r;
            const float2 yv = yv_[r];
            const double e = fma((double)v[r].y, (double)yv.x, -((double)v[r].x * (double)yv.y));   // Im(G^ conj(Y))
            const double ky = sfreq<N256>(ky_i) * dk;
            acc[0] = fma(e, fma(ky, ky, kx2), acc[0]);
            acc[1] = fma(e, kx, acc[1]);
            acc[2] = fma(e, ky, acc[2]);
            v[r] = cscale(tmul<true>(tmul<true>(v[r], tab.h[ky_i]), hx), inv_n2);
        }
        mid2nat<ColGeo256, +1>(v, lds, tab.tw, l, c);
        cols_store(v, w, x, c);
    } else {
        const float2* Pm = chain_probe(a, m, N256 * N256);
        float2* gP = a.gPhat + (size_t)ch * N256 * N256;
        const float2 rx = tab.rl[l];
        const double qx = (double)sfreq<N256>(x) / N256;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ky_i = c + 16 * r;
            const float2 G0 = cscale(v[r], inv_n);
            const float2 R = cmul(tab.r[ky_i], rx);
            gP[ky_i * N256 + x] = cmulc(G0, R);                          // conj(R) G^_0
            const float2 z = cmulc(cmul(Pm[ky_i * N256 + x], R), G0);    // Phat R conj(G^_0)
            acc[3] = fma((double)z.y, (double)sfreq<N256>(ky_i) / N256, acc[3]);
            acc[4] = fma((double)z.y, qx, acc[4]);
        }
    }
    block_sum<5>(acc, reinterpret_cast<double*>(lds));
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) part[k] += acc[k];
}

// Gradient row pass of slice s for P.mg consecutive chains of one position
// and object mode (probe modes p0 .. p0 + mg - 1): per chain the wave holds
// (y, k_x) of G after the inverse along y; the inverse along x gives
// G_chi_s, phi_s is rebuilt from the kept Z_s as the forward row pass formed
// it, the group's patch gradient sum_p conj(phi_s) G_chi (in probe-mode
// order) is summed in registers, and G_phi = conj(O_s) G_chi is transformed
// along x.  The object patch is read once for the group and the summed patch
// gradient written once, mg times less patch-gradient traffic (written here,
// read by the object scatter) than one per chain.  The next chain's phi_s is
// read while the current chain's line DFT runs.
__global__ __launch_bounds__(256) void k256_grad_row(Pass256 P) {
    __shared__ float2 lds[LDS256];
    __shared__ Tables256 tab;
    const WaveArgs& a = P.a;
    const int mg = P.mg, grp = a.chain0 / mg + blockIdx.x / NBLK256, blk = blockIdx.x % NBLK256;
    const int ch0 = grp * mg, j = ch0 / a.M;
    const PosInfo pi = a.pinfo[j];
    if (pi.ty < 0) return;
    const int l = threadIdx.x / 16, c = threadIdx.x % 16, y = blk * LINES256 + l;
    load256<1>(tab, P.tw, P.tab, j, blk * LINES256);
    float2 v[16], ph[16], ov[16], acc[16];
    rows_load(v, P.wave + (size_t)ch0 * N256 * N256, y, c);
    rows_load(ph, Slots<N256>(a, ch0).phi(P.s), y, c);
    // the object patch (the same for the group's chains) and the first
    // chain's G and phi_s are read now, so that their latency overlaps the
    // line DFT
    const float2* Os = chain_object(a, ch0 % a.M) + (size_t)P.s * a.H * a.W + (size_t)(pi.ty + y) * a.W + pi.tx;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        ov[r] = Os[c + 16 * r];
        acc[r] = make_float2(0.f, 0.f);
    }
    for (int p = 0; p < mg; ++p) {
        const int ch = ch0 + p;
        if (P.s == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) ph[r] = cmul(ph[r], tab.r[c + 16 * r]);
        }
        mid2nat<RowGeo256, +1>(ph, lds, tab.tw, l, c);                 // phi_s (space)
        mid2nat<RowGeo256, +1>(v, lds, tab.tw, l, c);                  // G_chi_s (space)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc[r] = cadd(acc[r], cmulc(v[r], ph[r]));                  // conj(phi) G_chi
            v[r] = cmulc(v[r], ov[r]);                                  // conj(O) G_chi
        }
        if (p + 1 < mg) rows_load(ph, Slots<N256>(a, ch + 1).phi(P.s), y, c);
        nat2mid<RowGeo256, -1>(v, lds, tab.tw, l, c);
        rows_store(v, P.wave + (size_t)ch * N256 * N256, y, c);
        if (p + 1 < mg) rows_load(v, P.wave + (size_t)(ch + 1) * N256 * N256, y, c);
    }
    float2* go = a.gO + (((size_t)grp * a.S + P.s) * N256 + y) * N256;
#pragma unroll
    for (int r = 0; r < 16; ++r) go[c + 16 * r] = acc[r];
}

// Orthonormal 2-D DFT of `count` 256 x 256 waves as two passes:
// rows (ROWS = true) then columns; the column pass scales by 1/256 and
// stores or accumulates.
template <int SG, bool ROWS, bool ACC>
__global__ __launch_bounds__(256) void k256_fft(const float2* in, float2* out) {
    __shared__ float2 lds[LDS256];
    __shared__ float4 tw[N256];
    const int wv = blockIdx.x / NBLK256, blk = blockIdx.x % NBLK256;
    {
        const int n = threadIdx.x;
        double s, c;
        sincos(-2.0 * 3.14159265358979323846 * (double)((n / 16) * (n % 16)) / N256, &s, &c);
        tw[n] = unit_pair(c, s);
    }
    __syncthreads();
    const float2* src = in + (size_t)wv * N256 * N256;
    float2* dst = out + (size_t)wv * N256 * N256;
    float2 v[16];
    if (ROWS) {
        const int l = threadIdx.x / 16, c = threadIdx.x % 16, y = blk * LINES256 + l;
        rows_load(v, src, y, c);
        nat2mid<RowGeo256, SG>(v, lds, tw, l, c);
        rows_store(v, dst, y, c);
    } else {
        const int l = threadIdx.x % 16, c = threadIdx.x / 16, x = blk * LINES256 + l;
        cols_load(v, src, x, c);
        nat2mid<ColGeo256, SG>(v, lds, tw, l, c);
        const float sc = 1.0f / N256;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float2 o = cscale(v[r], sc);
            if (ACC) o = cadd(o, dst[(c + 16 * r) * N256 + x]);
            v[r] = o;
        }
        cols_store(v, dst, x, c);
    }
}

}  // namespace ptyr
