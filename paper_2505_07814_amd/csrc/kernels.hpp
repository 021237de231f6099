// kernels.hpp - gfx950 kernels of the multislice forward model and its
// gradient.  One workgroup per (batch row, probe mode) keeps the whole N x N
// complex wave (N = 64 or 128) in registers across all slices and uses LDS
// only for line exchanges and transposes (wave.hpp).
//
// Per slice the forward takes the full 2-D spectrum of the transmitted wave,
// multiplies by the propagator and transforms back, so the spectrum of every
// incident wave, Y_s = F[phi_s], is formed on the way.  Kept for the gradient
// (when the memory budget allows): phi_s (space), Y_s (spectrum) and the
// far field.  The gradient kernel then holds a single wave in registers and
// streams those kept arrays element by element.  Kept waves, checkpoints and
// the recomputation scratch are written and read register-major (kstore /
// kload: register r of thread t at r T + t), in whatever register layout the
// wave has at that point, which the reading kernel knows.
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

// How the forward keeps waves for the gradient.
//   FULL : phi_s for every slice, Y_s for s >= 1, and the far field
//   CKPT : phi_s for s % ckK == 0 (ckK <= S) or nothing (ckK > S); the gradient
//          recomputes phi_s / Y_s into a 3-wave scratch per chain (phi, Y, G)
enum : int { KEEP_FULL = 0, KEEP_CKPT = 1 };

// Arguments shared by the fused forward / gradient kernels.
struct WaveArgs {
    const float2* Oc;      // S x H x W complex transmission a exp(i phase)
    const float2* Phat;    // M x N x N probe spectra F[P_m] (orthonormal)
    const PosInfo* pinfo;  // B, with validated rows
    const float* tilt;     // rows of (th_y, th_x)
    const float* dz;       // 1
    float2* store;         // kept waves, per chain: FULL 2S waves, CKPT nck + 3
    int keep;              // KEEP_FULL / KEEP_CKPT
    int ckK;               // checkpoint spacing (CKPT)
    int nck;               // checkpoints per chain (CKPT)
    int B, M, S, H, W;     // M: chain modes per row (probe modes x object modes)
    int Mp;                // probe modes: chain mode e uses probe mode e % Mp and object mode e / Mp
    size_t ostride;        // object-mode stride of Oc (S x H x W)
    int chain0;            // first chain (row * M + mode) of this launch; block b handles chain0 + b
    double dx, lam;
    int global_tilt;
    float* Imode;          // B x M x N x N, zero frequency at (0, 0)
    const float* wgt;      // B x N x N, 2 dL/dI, zero frequency at (0, 0)
    float2* gO;            // B x M x S x N x N object-patch gradients
    float2* gPhat;         // B x M x N x N probe-spectrum gradients
    double* part;          // B x M x 8 scalar partial sums (N = 256: per line block)
};

// probe spectrum and object transmission (all slices) of chain mode e
__device__ __forceinline__ const float2* chain_probe(const WaveArgs& a, int e, int NN) {
    return a.Phat + (size_t)(e % a.Mp) * NN;
}
__device__ __forceinline__ const float2* chain_object(const WaveArgs& a, int e) {
    return a.Oc + (size_t)(e / a.Mp) * a.ostride;
}

// Wave slots of one chain in the store.
template <int N> struct Slots {
    float2* base;
    int S, nck;
    __device__ Slots(const WaveArgs& a, int chain) : S(a.S), nck(a.nck) {
        const int per = a.keep == KEEP_FULL ? (N == 256 ? a.S + 1 : 2 * a.S) : a.nck + 3;
        base = a.store ? a.store + (size_t)chain * per * (N * N) : nullptr;
    }
    // FULL: [phi_0 .. phi_{S-1}] [Y_1 .. Y_{S-1}] [far field]; N = 256:
    // [Z_0 .. Z_{S-1}] [far field], Z_s the wave entering slice s's row pass
    __device__ float2* phi(int s) const { return base + (size_t)s * N * N; }
    __device__ float2* spec(int s) const { return base + (size_t)(S + s - 1) * N * N; }
    __device__ float2* far() const { return base + (size_t)(N == 256 ? S : 2 * S - 1) * N * N; }
    // CKPT: [checkpoints 0 .. nck-1] [scratch phi] [scratch Y] [scratch G]
    __device__ float2* ckpt(int k) const { return base + (size_t)k * N * N; }
    __device__ float2* sc_phi() const { return base + (size_t)nck * N * N; }
    __device__ float2* sc_spec() const { return base + (size_t)(nck + 1) * N * N; }
    __device__ float2* sc_g() const { return base + (size_t)(nck + 2) * N * N; }
};

// ------------------------------------------------------------------ tables
// Per-workgroup LDS tables: twiddles and the separable propagator factors.
template <int N> struct Tables {
    float4 tw[N];          // twiddles, b-major: tw[b*L + c] = exp(-2 pi i c b / N)
    float4 hy[N], hx[N];   // propagator factors along y (times 1/N^2) and x
    float2 ry[N], rx[N];   // shift ramp factors exp(-2 pi i q_n dr_y), exp(-2 pi i q_n dr_x)
};

template <int N>
__device__ __forceinline__ void build_tables(Tables<N>& t, const WaveArgs& a, const PosInfo& pi, float thy,
                                             float thx, float dz) {
    constexpr int T = N * N / 16;
    const double pi_d = 3.14159265358979323846;
    for (int i = threadIdx.x; i < 5 * N; i += T) {
        int which = i / N, n = i % N;
        double q = (double)sfreq<N>(n) / N;            // cycles per pixel
        double k = q / a.dx;                            // 1/angstrom
        double ph;
        if (which == 0) ph = -2.0 * pi_d * (double)((n / (N / 16)) * (n % (N / 16))) / N;
        else if (which == 1) ph = -pi_d * a.lam * dz * k * k + 2.0 * pi_d * dz * k * tan((double)thy);
        else if (which == 2) ph = -pi_d * a.lam * dz * k * k + 2.0 * pi_d * dz * k * tan((double)thx);
        else if (which == 3) ph = -2.0 * pi_d * q * pi.dry;
        else ph = -2.0 * pi_d * q * pi.drx;
        double s, c;
        sincos(ph, &s, &c);
        float4 w = unit_pair(c, s);
        if (which == 0) t.tw[n] = w;
        else if (which == 1) {   // the 1/N^2 of the two unnormalised transforms rides on h_y (exact: 2^-k)
            const float sc = 1.0f / ((float)N * N);
            t.hy[n] = make_float4(w.x * sc, w.y * sc, w.z * sc, w.w * sc);
        }
        else if (which == 2) t.hx[n] = w;
        else if (which == 3) t.ry[n] = make_float2(w.x, w.y);
        else t.rx[n] = make_float2(w.x, w.y);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ steps
// chi = O_s[t + (y, x)] * v  in layout (COL, NAT)
template <int N>
__device__ __forceinline__ void transmit(float2 (&v)[16], const float2* Os, int W, int ty, int tx, int l, int c) {
    using Y = Lay<N, COL, NAT>;
    const float2* base = Os + (size_t)ty * W + tx;
    const unsigned o = Y::toff(l, c, W);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        v[r] = cmul(v[r], (base + Y::dy(r) * W)[o]);
        if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
}

// the object patch O_s[t + (y, x)] in layout (COL, NAT)
template <int N>
__device__ __forceinline__ void load_patch(float2 (&ov)[16], const float2* Os, int W, int ty, int tx, int l, int c) {
    using Y = Lay<N, COL, NAT>;
    const float2* base = Os + (size_t)ty * W + tx;
    const unsigned o = Y::toff(l, c, W);
#pragma unroll
    for (int r = 0; r < 16; ++r) ov[r] = (base + Y::dy(r) * W)[o];
}

// phi_0 = F^-1[ Phat_m * R ] (orthonormal), leaves in (COL, NAT)
template <int N>
__device__ __forceinline__ void shift_probe(float2 (&v)[16], const float2* Pm, float2* lds, const Tables<N>& t,
                                            int l, int c) {
    const float sc = 1.0f / N;
    wload<N, ROW, MID>(v, Pm, N, l, c);
    const float2 ru = cscale(t.ry[l], sc);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cmul(cmul(v[r], ru), t.rx[line_pos<N, MID>(c, r)]);
    mid2nat<WaveGeo<N>, +1>(v, lds, t.tw, l, c);
    relayout<N, ROW, NAT, COL, MID>(v, lds, l, c);
    mid2nat<WaveGeo<N>, +1>(v, lds, t.tw, l, c);
}

// unnormalised 2-D DFT of sign -1 from (COL, NAT); leaves in (ROW, MID)
template <int N>
__device__ __forceinline__ void fft2_from_col(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    nat2mid<WaveGeo<N>, -1>(v, lds, tw, l, c);
    relayout<N, COL, MID, ROW, NAT>(v, lds, l, c);
    nat2mid<WaveGeo<N>, -1>(v, lds, tw, l, c);
}
// unnormalised 2-D inverse DFT from (ROW, MID); leaves in (COL, NAT)
template <int N>
__device__ __forceinline__ void ifft2_to_col(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    mid2nat<WaveGeo<N>, +1>(v, lds, tw, l, c);
    relayout<N, ROW, NAT, COL, MID>(v, lds, l, c);
    mid2nat<WaveGeo<N>, +1>(v, lds, tw, l, c);
}

// Multiply a (ROW, MID) spectrum by H / N^2 (or conj(H) / N^2); the table h_y
// carries the 1/N^2.
template <int N, bool CONJ>
__device__ __forceinline__ void apply_h(float2 (&v)[16], const Tables<N>& t, int l, int c) {
    const float4 hy = t.hy[l];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        v[r] = tmul<CONJ>(tmul<CONJ>(v[r], hy), t.hx[line_pos<N, MID>(c, r)]);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

// One slice step: v = phi_s (COL, NAT) -> chi_s -> (F, H, F^-1) -> phi_{s+1}
// (COL, NAT).  The spectrum Y'_{s+1} = H F_raw[chi_s] / N^2 = F_raw[phi_{s+1}] / N^2
// is written to spec when spec != nullptr.
template <int N>
__device__ __forceinline__ void slice_step(float2 (&v)[16], const float2* Os, int W, int ty, int tx, float2* spec,
                                           float2* lds, const Tables<N>& t, int l, int c) {
    transmit<N>(v, Os, W, ty, tx, l, c);
    fft2_from_col<N>(v, lds, t.tw, l, c);
    apply_h<N, false>(v, t, l, c);
    if (spec) kstore<N>(v, spec);
    ifft2_to_col<N>(v, lds, t.tw, l, c);
}

// block-wide sum of NV values, result valid in thread 0
template <int NV, typename T>
__device__ __forceinline__ void block_sum(T (&x)[NV], T* red) {
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
            T s = 0;
            for (int q = 0; q < nw; ++q) s += red[q * NV + k];
            x[k] = s;
        }
    __syncthreads();
}

// ------------------------------------------------------------------ kernels
// LDS slots the forward declares.  At N = 128 it uses half of the compute
// unit's 160 KiB but reserves all of it: small kernels launched beside the
// forward (the loss rows of the first chain range) then run on free compute
// units instead of sharing the forward's, where they would stretch out
// behind its waves (measured: 67 -> 28 us for those loss rows).
template <int N> constexpr int fwd_lds_slots() {
    return N == 128 ? (int)((160 * 1024 - sizeof(Tables<N>)) / sizeof(float2)) : WaveGeo<N>::LDS_SLOTS;
}

// Forward: one workgroup per (batch row j, probe mode m).  KEEP (the wave
// store plan) is a template parameter so that the hot loop has no
// data-dependent branch around its writes: at such a merge the compiler's
// wait for the object-patch reads would also wait for the writes.
template <int N, int KEEP>
__global__ __launch_bounds__(N * N / 16) void k_forward(WaveArgs a) {
    __shared__ float2 lds[fwd_lds_slots<N>()];
    __shared__ Tables<N> tab;
    int l, c;
    line_of<N>(threadIdx.x, l, c);
    const int wg = a.chain0 + xcd_remap(blockIdx.x, gridDim.x);
    const int j = wg / a.M, m = wg % a.M;
    const PosInfo pi = a.pinfo[j];
    float* Iout = a.Imode + (size_t)(j * a.M + m) * N * N;
    if (pi.ty < 0) {
        for (int i = threadIdx.x; i < N * N; i += blockDim.x) Iout[i] = 0.f;
        return;
    }
    const float* th = a.global_tilt ? a.tilt : a.tilt + 2 * pi.row;
    build_tables<N>(tab, a, pi, th[0], th[1], *a.dz);
    const Slots<N> sl(a, j * a.M + m);
    constexpr bool full = KEEP == KEEP_FULL;            // the store is always in the workspace
    const bool ckpt = KEEP == KEEP_CKPT && a.ckK <= a.S;
    const size_t HW = (size_t)a.H * a.W;

    const float2* Ocm = chain_object(a, m);
    float2 v[16];
    shift_probe<N>(v, chain_probe(a, m, N * N), lds, tab, l, c);
    // the object patch of a slice is read one slice ahead, so that its
    // latency overlaps the previous slice's transforms (forward launch
    // 0.486 -> 0.467 ms)
    float2 ov[16];
    if (a.S > 1) load_patch<N>(ov, Ocm, a.W, pi.ty, pi.tx, l, c);
    for (int s = 0; s < a.S - 1; ++s) {
        // chi_s is formed in ov before phi_s is written: waiting for the patch
        // then cannot wait for those (conditional) writes as well.  v keeps
        // phi_s while ov is transformed, and the kept waves are written in
        // groups spaced by the transforms' stages (phi_s in quarters, Y_s in
        // halves), so that a wave's writes do not queue up all at once behind
        // those of the other waves.
#pragma unroll
        for (int r = 0; r < 16; ++r) ov[r] = cmul(v[r], ov[r]);
        if (full) kstore_q<N, 0>(v, sl.phi(s));
        else if (ckpt && s % a.ckK == 0) kstore<N>(v, sl.ckpt(s / a.ckK));
        __builtin_amdgcn_sched_barrier(0);
        nat2mid<WaveGeo<N>, -1>(ov, lds, tab.tw, l, c);
        __builtin_amdgcn_sched_barrier(0);
        if (full) kstore_q<N, 1>(v, sl.phi(s));
        __builtin_amdgcn_sched_barrier(0);
        relayout<N, COL, MID, ROW, NAT>(ov, lds, l, c);
        __builtin_amdgcn_sched_barrier(0);
        if (full) kstore_q<N, 2>(v, sl.phi(s));
        __builtin_amdgcn_sched_barrier(0);
        nat2mid<WaveGeo<N>, -1>(ov, lds, tab.tw, l, c);
        __builtin_amdgcn_sched_barrier(0);
        if (full) kstore_q<N, 3>(v, sl.phi(s));
        apply_h<N, false>(ov, tab, l, c);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ov[r];
        if (full) kstore_half<N, 0>(ov, sl.spec(s + 1));
        __builtin_amdgcn_sched_barrier(0);
        mid2nat<WaveGeo<N>, +1>(v, lds, tab.tw, l, c);
        __builtin_amdgcn_sched_barrier(0);
        if (full) kstore_half<N, 1>(ov, sl.spec(s + 1));
        relayout<N, ROW, NAT, COL, MID>(v, lds, l, c);
        if (s + 1 < a.S - 1) load_patch<N>(ov, Ocm + (size_t)(s + 1) * HW, a.W, pi.ty, pi.tx, l, c);
        mid2nat<WaveGeo<N>, +1>(v, lds, tab.tw, l, c);
    }
    const int s = a.S - 1;
    if (full) kstore<N>(v, sl.phi(s));
    else if (ckpt && s % a.ckK == 0) kstore<N>(v, sl.ckpt(s / a.ckK));
    transmit<N>(v, Ocm + (size_t)s * HW, a.W, pi.ty, pi.tx, l, c);
    fft2_from_col<N>(v, lds, tab.tw, l, c);
    if (full) kstore<N>(v, sl.far());
    // far field |F chi|^2 / N^2 (zero frequency at (0, 0); the mode sum shifts it)
    const float s2 = 1.0f / ((float)N * N);
    float iv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) iv[r] = cabs2(v[r]) * s2;
    wstore<N, ROW, MID>(iv, Iout, N, l, c);
}

// Recompute phi_s (COL, NAT) with the forward's own slice steps, starting
// from the last kept checkpoint at or before slice s-1 (or from the shifted
// probe when none is kept), so that for s > 0 the last step also yields
// Y'_s, written to spec.  Recomputed values are bitwise those of the forward.
template <int N>
__device__ __forceinline__ void recompute_phi(float2 (&v)[16], int s, const WaveArgs& a, const Slots<N>& sl, int m,
                                              int ty, int tx, float2* spec, float2* lds, const Tables<N>& t, int l,
                                              int c) {
    int s0 = 0;
    if (a.ckK <= a.S) {
        s0 = s > 0 ? ((s - 1) / a.ckK) * a.ckK : 0;
        kload<N>(v, sl.ckpt(s0 / a.ckK));
    } else {
        shift_probe<N>(v, chain_probe(a, m, N * N), lds, t, l, c);
    }
    const size_t HW = (size_t)a.H * a.W;
    const float2* Ocm = chain_object(a, m);
    for (int u = s0; u < s; ++u)
        slice_step<N>(v, Ocm + (size_t)u * HW, a.W, ty, tx, u == s - 1 ? spec : nullptr, lds, t, l, c);
}

// Gradient: one workgroup per (batch row j, probe mode m).  Walks the slices
// backwards (chain rule through Eq. 2-4) holding only the adjoint field G in
// registers; phi_s, Y_s and the far field are streamed from the store
// (KEEP = KEEP_FULL) or recomputed into the chain's scratch (KEEP_CKPT).
// Writes per-slice object-patch gradients conj(phi_s) G_chi, the
// probe-spectrum gradient conj(R) G^_0 and partial sums for the position,
// tilt and dz gradients.
template <int N, int KEEP>
__global__ __launch_bounds__(N * N / 16) void k_gradient(WaveArgs a) {
    constexpr int T = N * N / 16;
    __shared__ float2 lds[WaveGeo<N>::LDS_SLOTS];
    __shared__ Tables<N> tab;
    int l, c;
    line_of<N>(threadIdx.x, l, c);
    const int wg = a.chain0 + xcd_remap(blockIdx.x, gridDim.x);
    const int j = wg / a.M, m = wg % a.M;
    const PosInfo pi = a.pinfo[j];
    double* part = a.part + (size_t)(j * a.M + m) * 8;
    float2* gP = a.gPhat + (size_t)(j * a.M + m) * N * N;
    if (pi.ty < 0) {
        for (int i = threadIdx.x; i < N * N; i += blockDim.x) gP[i] = make_float2(0.f, 0.f);
        if (threadIdx.x < 8) part[threadIdx.x] = 0.0;
        return;   // the object-gradient scatter skips such rows
    }
    const float* th = a.global_tilt ? a.tilt : a.tilt + 2 * pi.row;
    build_tables<N>(tab, a, pi, th[0], th[1], *a.dz);
    const Slots<N> sl(a, j * a.M + m);
    const size_t HW = (size_t)a.H * a.W;
    const float inv_n = 1.0f / N, inv_n2 = 1.0f / ((float)N * N);

    float2 g[16];
    // far field: kept, or recomputed from phi_{S-1}
    if (KEEP == KEEP_FULL) {
        kload<N>(g, sl.far());
    } else {
        recompute_phi<N>(g, a.S - 1, a, sl, m, pi.ty, pi.tx, sl.sc_spec(), lds, tab, l, c);
        transmit<N>(g, chain_object(a, m) + (size_t)(a.S - 1) * HW, a.W, pi.ty, pi.tx, l, c);
        fft2_from_col<N>(g, lds, tab.tw, l, c);
    }
    {   // G_chi_{S-1} = F^-1[ w F[chi_{S-1}] ]   (w = 2 dL/dI)
        float wv[16];
        wload<N, ROW, MID>(wv, a.wgt + (size_t)j * N * N, N, l, c);
#pragma unroll
        for (int r = 0; r < 16; ++r) g[r] = cscale(g[r], wv[r] * inv_n2);
    }
    ifft2_to_col<N>(g, lds, tab.tw, l, c);

    using YC = Lay<N, COL, NAT>;
    using YR = Lay<N, ROW, MID>;
    const unsigned oW = YC::toff(l, c, a.W);
    const unsigned oM = YR::toff(l, c, N);

    // chi_s = O_s phi_s: gO_s = conj(phi_s) G_chi, then G_phi = conj(O_s) G_chi,
    // then G^ = F_raw G_phi.  Returns the stream of Y'_s for s > 0.
    auto slice_back = [&](int s) -> const float2* {
        const float2 *phi_s, *Y_s;
        if (KEEP == KEEP_FULL) {
            phi_s = sl.phi(s);
            Y_s = s > 0 ? sl.spec(s) : nullptr;
        } else {
            // park G, recompute phi_s and Y'_s into the scratch, take G back
            kstore<N>(g, sl.sc_g());
            recompute_phi<N>(g, s, a, sl, m, pi.ty, pi.tx, sl.sc_spec(), lds, tab, l, c);
            kstore<N>(g, sl.sc_phi());
            kload<N>(g, sl.sc_g());
            phi_s = sl.sc_phi();
            Y_s = sl.sc_spec();
        }
        const float2* Os = chain_object(a, m) + (size_t)s * HW + (size_t)pi.ty * a.W + pi.tx;
        float2* go = a.gO + ((size_t)(j * a.M + m) * a.S + s) * N * N;
        // The patch gradient is stored register-major (register r of thread t
        // at r T + t, T threads: each store instruction writes one contiguous
        // 512-byte run per wave; the scatter maps pixels to that order,
        // measured 0.419 -> 0.406 ms per launch against row-major stores).
        // The reads run in two halves of 8 registers (32 VGPRs in flight),
        // each issued before any patch-gradient write that follows it: the
        // writes could alias the reads as far as the compiler knows, and one
        // in-order counter covers reads and writes, so a read issued after a
        // write waits for that write too.  Half 0's patch gradient t0 is
        // therefore written only after half 1's reads are issued (measured:
        // gradient launch 0.432 -> 0.417 ms).
        float2 t0[8], t1[4];
        {
            float2 ph[8], ov[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                ph[r] = (phi_s + r * T)[threadIdx.x];
                ov[r] = (Os + YC::dy(r) * a.W)[oW];
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                t0[r] = cmulc(g[r], ph[r]);                                    // conj(phi) G_chi
                g[r] = cmulc(g[r], ov[r]);                                     // G_phi = conj(O) G_chi
            }
        }
        {
            float2 ph[8], ov[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                ph[r] = (phi_s + (8 + r) * T)[threadIdx.x];
                ov[r] = (Os + YC::dy(8 + r) * a.W)[oW];
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (r < 4) t1[r] = cmulc(g[8 + r], ph[r]);
                else (go + (8 + r) * T)[threadIdx.x] = cmulc(g[8 + r], ph[r]);
                g[8 + r] = cmulc(g[8 + r], ov[r]);
            }
        }
        // G^ = F_raw G_phi; the patch gradient's quarters 0 and 2 (t0[0..3],
        // t1) are written after the first line pass and quarter 1 after the
        // exchange (quarter 3 went out before the transform), so that the
        // chain's writes come in spaced groups
        __builtin_amdgcn_sched_barrier(0);
        nat2mid<WaveGeo<N>, -1>(g, lds, tab.tw, l, c);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) (go + r * T)[threadIdx.x] = t0[r];
#pragma unroll
        for (int r = 0; r < 4; ++r) (go + (8 + r) * T)[threadIdx.x] = t1[r];
        __builtin_amdgcn_sched_barrier(0);
        relayout<N, COL, MID, ROW, NAT>(g, lds, l, c);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 4; r < 8; ++r) (go + r * T)[threadIdx.x] = t0[r];
        nat2mid<WaveGeo<N>, -1>(g, lds, tab.tw, l, c);
        return Y_s;
    };

    // dz / tilt / position partial sums in double: Im(G^ conj(Y)) is formed
    // from the exact double products of the float values, and the sums over
    // registers, slices and threads carry no float rounding (the dz gradient
    // is a sum of terms of both signs)
    double acc_k2 = 0.0, acc_kx = 0.0, acc_ky = 0.0;
    const double dk = 1.0 / (N * a.dx);
    const double ky = sfreq<N>(l) * dk, ky2 = ky * ky;
    for (int s = a.S - 1; s >= 1; --s) {
        const float2* Y_s = slice_back(s);
        // dL/d(dz, th) += sum_k dPhi/dt(k) Im(G^ conj(Y)), Y = F phi_s (raw G^ x Y')
        // Y is read in one batch; the per-register k_x are recomputed each
        // slice (the opaque copy of the lane index keeps the compiler from
        // hoisting all sixteen out of the loop into spills)
        int cc = c;
        asm volatile("" : "+v"(cc));
        float2 yv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) yv[r] = (Y_s + r * T)[threadIdx.x];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float2 y = yv[r];
            const double e = fma((double)g[r].y, (double)y.x, -((double)g[r].x * (double)y.y));
            const double kx = sfreq<N>(line_pos<N, MID>(cc, r)) * dk;
            acc_k2 = fma(e, fma(kx, kx, ky2), acc_k2);
            acc_kx = fma(e, kx, acc_kx);
            acc_ky = fma(e, ky, acc_ky);
        }
        apply_h<N, true>(g, tab, l, c);                                       // conj(H) G^ / N^2
        ifft2_to_col<N>(g, lds, tab.tw, l, c);                                // G_chi_{s-1}
    }
    slice_back(0);
    // probe spectrum and position: phi_0 = F^-1[Phat R]
    double acc_py = 0.0, acc_px = 0.0;
    {
        const float2* Pm = chain_probe(a, m, N * N);
        const float2 ry = tab.ry[l];
        const double qy = (double)sfreq<N>(l) / N;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int x = line_pos<N, MID>(c, r);
            const float2 G0 = cscale(g[r], inv_n);
            const float2 R = cmul(ry, tab.rx[x]);
            g[r] = cmulc(G0, R);                                               // conj(R) G^_0
            const float2 z = cmulc(cmul((Pm + YR::dx(r))[oM], R), G0);         // Phat R conj(G^_0)
            acc_py = fma((double)z.y, qy, acc_py);
            acc_px = fma((double)z.y, (double)sfreq<N>(x) / N, acc_px);
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        wstore<N, ROW, MID>(g, gP, N, l, c);
    }
    double sums[5] = {acc_k2, acc_kx, acc_ky, acc_py, acc_px};
    block_sum<5>(sums, reinterpret_cast<double*>(lds));  // the transpose buffer is free again
    if (threadIdx.x == 0) {
        for (int k = 0; k < 5; ++k) part[k] = sums[k];
        part[5] = part[6] = part[7] = 0.0;
    }
}

// One N x N 2-D DFT of sign SG by a whole workgroup (N*N/16 threads), scaled
// by 1/N (orthonormal); the result is written to dst, or added to it (ACC).
template <int N, int SG, bool ACC>
__device__ __forceinline__ void fft2_block(const float2* src, float2* dst) {
    __shared__ float2 lds[WaveGeo<N>::LDS_SLOTS];
    __shared__ float4 tw[N];
    int l, c;
    line_of<N>(threadIdx.x, l, c);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        double s, co;
        sincos(-2.0 * 3.14159265358979323846 * (double)((n / (N / 16)) * (n % (N / 16))) / N, &s, &co);
        tw[n] = unit_pair(co, s);
    }
    __syncthreads();
    float2 v[16];
    wload<N, ROW, NAT>(v, src, N, l, c);
    nat2mid<WaveGeo<N>, SG>(v, lds, tw, l, c);
    relayout<N, ROW, MID, COL, NAT>(v, lds, l, c);
    nat2mid<WaveGeo<N>, SG>(v, lds, tw, l, c);
    const float sc = 1.0f / N;
    float2 o[16];
    if (ACC) wload<N, COL, MID>(o, dst, N, l, c);
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = ACC ? cadd(cscale(v[r], sc), o[r]) : cscale(v[r], sc);
    wstore<N, COL, MID>(o, dst, N, l, c);
}

// the 2-D DFT of each of gridDim.x fields (one workgroup each)
template <int N, int SG, bool ACC>
__global__ __launch_bounds__(N * N / 16) void k_fft2(const float2* in, float2* out) {
    fft2_block<N, SG, ACC>(in + (size_t)blockIdx.x * N * N, out + (size_t)blockIdx.x * N * N);
}

}  // namespace ptyr
