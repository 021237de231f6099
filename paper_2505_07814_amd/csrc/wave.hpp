// wave.hpp - register-resident N x N complex wave for one workgroup (gfx950).
//
// A workgroup of T = N*N/16 threads holds one N x N complex64 field, 16
// values per thread.  The field is seen as N "lines" (rows or columns); a
// line is owned by L = N/16 consecutive lanes.  Two register layouts of a
// line are used (c = lane within the line, r = register 0..15):
//
//   NAT : register r holds line element  n = c + L*r
//   MID : register r = beta*L + a holds  n = (c + L*beta) + 16*a
//
// A length-N DFT along the lines is split as N = 16 * L:
//   nat2mid: 16-point DFT in registers, twiddle W_N^{c b}, exchange,
//            L-point DFT in registers            (NAT in -> MID out)
//   mid2nat: the same factors in reverse order   (MID in -> NAT out)
// The exchange between the two DFTs transposes, in every line, L x L blocks
// of registers against the line's L lanes.  For N = 64 and 128 the L lanes of
// a line sit 64 / L lanes apart in one wave (line_of), so the transpose's
// butterfly stages pair lanes 16 and 32 (and, for L = 8, 8) apart and run as
// cross-lane register swaps (v_permlane16_swap / v_permlane32_swap, and a
// masked DPP row rotation): no LDS traffic and no wait.  Line geometries
// without that placement (the N = 256 line passes) exchange through LDS.
// Either direction can carry either sign, so a line FFT, a pointwise
// multiply in frequency and a line IFFT keep the field in place.  A
// transpose (rows <-> columns) goes through LDS.  LDS slots are padded
// linear maps (slot = base(thread) + constant(register)), so every access is
// one base register plus an immediate offset; the paddings make LDS line
// exchanges bank-conflict free for each 32-lane half-wave and leave the
// transpose reads at most 2-way conflicted.  Transforms are unnormalised;
// callers fold the 1/N factors into their pointwise factors.
#pragma once
#include <hip/hip_runtime.h>

namespace ptyr {

// ------------------------------------------------------------ complex math
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }
// multiply by SG*i  (SG = +1 or -1)
template <int SG> __device__ __forceinline__ float2 mul_si(float2 a) {
    return SG > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// Constant twiddles are applied with compensated ("double-float") constants:
// c = c_hi + c_lo with c_hi the float nearest c.  A plain float constant such
// as float(sqrt(1/2)) has |w| = 1 - 1.7e-8, and because the same constants
// are hit on every pass of every slice that bias would add up linearly over
// the slices; the compensated product keeps the error of each multiply
// unbiased at the half-ulp level.
struct KC {
    float hi, lo;
};
constexpr KC kc(double v) { return KC{(float)v, (float)(v - (double)(float)v)}; }
constexpr KC RSQ2 = kc(0.70710678118654752440);   // cos(pi/4)
constexpr KC C8 = kc(0.92387953251128675613);     // cos(pi/8)
constexpr KC S8 = kc(0.38268343236508977173);     // sin(pi/8)

__device__ __forceinline__ float kmul(float x, KC c) { return fmaf(x, c.hi, x * c.lo); }
// x * c + y * d with compensated constants
__device__ __forceinline__ float kdot(float x, KC c, float y, KC d) {
    return fmaf(x, c.hi, fmaf(y, d.hi, fmaf(x, c.lo, y * d.lo)));
}
// (x + i y) * (cr + i ci) for compensated constants; ncr / nci negate the parts
template <bool NCR, bool NCI>
__device__ __forceinline__ float2 kcmul(float2 a, KC cr, KC ci) {
    KC r = NCR ? KC{-cr.hi, -cr.lo} : cr;
    KC i = NCI ? KC{-ci.hi, -ci.lo} : ci;
    KC mi = KC{-i.hi, -i.lo};
    return make_float2(kdot(a.x, r, a.y, mi), kdot(a.x, i, a.y, r));
}
// multiply by exp(SG * 2 pi i m / 16) for the twiddles m the 16-point DFT uses
template <int SG> __device__ __forceinline__ float2 tw16(float2 a, int m) {
    constexpr bool NEG = SG < 0;
    switch (m & 15) {
        case 1: return kcmul<false, NEG>(a, C8, S8);            // ( c8,  s8)
        case 2: return kcmul<false, NEG>(a, RSQ2, RSQ2);        // ( r,   r )
        case 3: return kcmul<false, NEG>(a, S8, C8);            // ( s8,  c8)
        case 4: return mul_si<SG>(a);                           // ( 0,   1 )
        case 6: return kcmul<true, NEG>(a, RSQ2, RSQ2);         // (-r,   r )
        case 9: return kcmul<true, !NEG>(a, C8, S8);            // (-c8, -s8)
        default: return a;
    }
}

// Round a unit complex number given in double to the float pair (one of the
// four neighbouring roundings) whose modulus is closest to 1.  Table factors
// applied on every slice (twiddles, propagator) would otherwise carry a
// fixed per-entry modulus error that compounds over the slices.
__device__ __forceinline__ float2 unit_round(double c, double s) {
    float c0 = (float)c, s0 = (float)s;
    float c1 = ((double)c0 > c) ? nextafterf(c0, -2.0f) : nextafterf(c0, 2.0f);
    float s1 = ((double)s0 > s) ? nextafterf(s0, -2.0f) : nextafterf(s0, 2.0f);
    float cs[2] = {c0, c1}, ss[2] = {s0, s1};
    float2 best = make_float2(c0, s0);
    double be = fabs((double)c0 * c0 + (double)s0 * s0 - 1.0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double e = fabs((double)cs[i] * cs[i] + (double)ss[j] * ss[j] - 1.0);
            if (e < be) { be = e; best = make_float2(cs[i], ss[j]); }
        }
    return best;
}

// ------------------------------------------------------------ small DFTs
template <int SG> __device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d) {
    float2 y0 = cadd(a, c), y1 = csub(a, c), y2 = cadd(b, d), y3 = mul_si<SG>(csub(b, d));
    a = cadd(y0, y2);
    c = csub(y0, y2);
    b = cadd(y1, y3);
    d = csub(y1, y3);
}

template <int SG> __device__ __forceinline__ void dft8(float2* x) {
    float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4<SG>(e0, e1, e2, e3);
    dft4<SG>(o0, o1, o2, o3);
    // W8^1 = r (1 + SG i), W8^3 = r (-1 + SG i), r = sqrt(1/2)
    o1 = make_float2(kmul(o1.x - SG * o1.y, RSQ2), kmul(SG * o1.x + o1.y, RSQ2));
    o2 = mul_si<SG>(o2);
    o3 = make_float2(kmul(-o3.x - SG * o3.y, RSQ2), kmul(SG * o3.x - o3.y, RSQ2));
    x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
    x[1] = cadd(e1, o1); x[5] = csub(e1, o1);
    x[2] = cadd(e2, o2); x[6] = csub(e2, o2);
    x[3] = cadd(e3, o3); x[7] = csub(e3, o3);
}

// 16-point DFT in natural order, 4 x 4 split: X[k1 + 4 k2] =
// sum_n2 W16^{n2 k1} W4^{n2 k2} sum_n1 x[4 n1 + n2] W4^{n1 k1}
template <int SG> __device__ __forceinline__ void dft16(float2* x) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<SG>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2]);
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) x[4 * k1 + n2] = tw16<SG>(x[4 * k1 + n2], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<SG>(x[4 * k1], x[4 * k1 + 1], x[4 * k1 + 2], x[4 * k1 + 3]);
    float2 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = x[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = t[i];
}

template <int L, int SG> __device__ __forceinline__ void dftL(float2* x) {
    static_assert(L == 4 || L == 8 || L == 16, "lanes per line must be 4, 8 or 16");
    if constexpr (L == 4) dft4<SG>(x[0], x[1], x[2], x[3]);
    else if constexpr (L == 8) dft8<SG>(x);
    else dft16<SG>(x);
}

// ------------------------------------------------------------ layouts
enum { ROW = 0, COL = 1 };
enum { NAT = 0, MID = 1 };

template <int N> struct WaveGeo {
    static constexpr int NL = N;          // line length
    static constexpr int L = N / 16;
    static constexpr int T = N * N / 16;
    static constexpr int G = 16 / L;
    // N = 128 halves the buffer (80 KiB with the tables): a line exchange
    // runs as two rounds of 8 registers, and a transpose moves the real
    // parts, then the imaginary parts, through a float buffer.  Measured on
    // gfx950 this is a few per cent faster than the full-size exchange, and
    // it would let two workgroups share a compute unit.
    static constexpr bool HALF = (N == 128);
    // LDS paddings: exchange element (line l, b, lane c) at float2 slot
    // l*SL + b*SB + c (b < 8 when HALF); field element (y, x) at float2 slot
    // y*SY + x, or (HALF) at float y*SYF + x.
    static constexpr int SB = (N == 128) ? 9 : 5;
    static constexpr int SL = (N == 128) ? 72 : 100;
    static constexpr int SY = N + L;
    static constexpr int SYF = N + L;
    static constexpr int XCH_SLOTS = (N - 1) * SL + (HALF ? 7 : 15) * SB + L;
    static constexpr int T_SLOTS = HALF ? (N * SYF + 1) / 2 : N * SY;
    static constexpr int LDS_SLOTS = XCH_SLOTS > T_SLOTS ? XCH_SLOTS : T_SLOTS;
    static constexpr bool WAVE_LOCAL = true;      // a line's lanes share a wave
    static constexpr bool XLANE = true;           // line exchanges by cross-lane swaps (line_of placement)
};

// (line l, lane c within the line) of thread tid for WaveGeo<N>: the wave
// holds 64 / L lines, and lane c of its k-th line is wave lane k + (64 / L) c
template <int N> __device__ __forceinline__ void line_of(int tid, int& l, int& c) {
    constexpr int L = N / 16, LPW = 64 / L;
    const int w = tid >> 6, ln = tid & 63;
    l = w * LPW + ln % LPW;
    c = ln / LPW;
}

// geometry traits with defaults for line geometries that do not set them
template <class GEO, class = void> struct HalfX {
    static constexpr bool value = false;
};
template <class GEO> struct HalfX<GEO, decltype(void(GEO::HALF))> {
    static constexpr bool value = GEO::HALF;
};
template <class GEO, class = void> struct XLaneX {
    static constexpr bool value = false;
};
template <class GEO> struct XLaneX<GEO, decltype(void(GEO::XLANE))> {
    static constexpr bool value = GEO::XLANE;
};

// position along the line of register r
template <int N, int K> __device__ __forceinline__ int line_pos(int c, int r) {
    constexpr int L = N / 16;
    if constexpr (K == NAT) return c + L * r;
    else return (c + L * (r / L)) + 16 * (r % L);
}

// (y, x) of register r of thread (line l, lane c)
template <int N, int D, int K> __device__ __forceinline__ void reg_yx(int l, int c, int r, int& y, int& x) {
    int n = line_pos<N, K>(c, r);
    if constexpr (D == ROW) { y = l; x = n; }
    else { y = n; x = l; }
}

// Affine split of a register's (y, x): y = yl + dy(r), x = xl + dx(r), with
// (yl, xl) the thread part and (dy, dx) a compile-time register part, so an
// element at row stride S sits at  [thread: yl*S + xl] + [uniform: dy*S + dx].
// Memory accesses use that form (one 32-bit thread offset plus a scalar base
// per register) instead of a 64-bit address per register.
template <int N, int D, int K> struct Lay {
    static constexpr int L = N / 16;
    static constexpr int n_of(int r) { return K == NAT ? L * r : L * (r / L) + 16 * (r % L); }
    static constexpr int dy(int r) { return D == ROW ? 0 : n_of(r); }
    static constexpr int dx(int r) { return D == ROW ? n_of(r) : 0; }
    __device__ static int yl(int l, int c) { return D == ROW ? l : c; }
    __device__ static int xl(int l, int c) { return D == ROW ? c : l; }
    __device__ static unsigned toff(int l, int c, int stride) { return (unsigned)(yl(l, c) * stride + xl(l, c)); }
};

template <int N, int D, int K, typename T>
__device__ __forceinline__ void wload(T (&v)[16], const T* base, int stride, int l, int c) {
    using Y = Lay<N, D, K>;
    const unsigned o = Y::toff(l, c, stride);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = (base + (Y::dy(r) * stride + Y::dx(r)))[o];
}
template <int N, int D, int K, typename T>
__device__ __forceinline__ void wstore(const T (&v)[16], T* base, int stride, int l, int c) {
    using Y = Lay<N, D, K>;
    const unsigned o = Y::toff(l, c, stride);
#pragma unroll
    for (int r = 0; r < 16; ++r) (base + (Y::dy(r) * stride + Y::dx(r)))[o] = v[r];
}

// A wave kept in device memory for the same workgroup geometry to read back
// (the kept waves, checkpoints and scratch of the fused kernels): register r
// of thread t at r T + t, T = N^2 / 16 threads, so every access instruction
// moves one contiguous 512-byte run per wave whatever the register layout.
template <int N, typename T> __device__ __forceinline__ void kstore(const T (&v)[16], T* base) {
    constexpr int TT = N * N / 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) (base + r * TT)[threadIdx.x] = v[r];
}
// registers 8 H .. 8 H + 7 only
template <int N, int H, typename T> __device__ __forceinline__ void kstore_half(const T (&v)[16], T* base) {
    constexpr int TT = N * N / 16;
#pragma unroll
    for (int r = 8 * H; r < 8 * H + 8; ++r) (base + r * TT)[threadIdx.x] = v[r];
}
template <int N, int Q, typename T> __device__ __forceinline__ void kstore_q(const T (&v)[16], T* base) {
    constexpr int TT = N * N / 16;
#pragma unroll
    for (int r = 4 * Q; r < 4 * Q + 4; ++r) (base + r * TT)[threadIdx.x] = v[r];
}
template <int N, typename T> __device__ __forceinline__ void kload(T (&v)[16], const T* base) {
    constexpr int TT = N * N / 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = (base + r * TT)[threadIdx.x];
}

// LDS slot of exchange element (line l, b, lane c') for line geometry GEO
// (GEO::L lanes per line, paddings GEO::SB, GEO::SL)
template <class GEO> __device__ __forceinline__ int slot_x(int l, int b, int c) {
    return l * GEO::SL + b * GEO::SB + c;
}

// LDS slot of field element (y, x) for a transpose
template <int N> __device__ __forceinline__ int slot_t(int y, int x) { return y * WaveGeo<N>::SY + x; }

// Table factors are kept as compensated pairs (hi, lo) in one float4:
// w = (x + z) + i (y + w).  Their product with a value is unbiased at the
// half-ulp level, so the fixed table entries applied on every pass of every
// slice do not add up a systematic modulus error.
__device__ __forceinline__ float4 unit_pair(double c, double s) {
    float2 h = unit_round(c, s);
    return make_float4(h.x, h.y, (float)(c - (double)h.x), (float)(s - (double)h.y));
}
// a * w  (CONJ: a * conj(w)) for a compensated table factor w
template <bool CONJ> __device__ __forceinline__ float2 tmul(float2 a, float4 w) {
    float wi = CONJ ? -w.y : w.y, li = CONJ ? -w.w : w.w;
    return make_float2(fmaf(a.x, w.x, fmaf(-a.y, wi, fmaf(a.x, w.z, -a.y * li))),
                       fmaf(a.x, wi, fmaf(a.y, w.x, fmaf(a.x, li, a.y * w.z))));
}

// v[b] *= W_N^{SG c b} for b = 1..15 from the compensated table, stored
// b-major (tw[b*L + c]) so that the lanes of a wave read consecutive entries.
// Scheduling fences keep at most four table entries (16 VGPRs) in flight;
// left alone the scheduler hoists all fifteen 128-bit reads.
template <int L, int SG> __device__ __forceinline__ void twiddle_pass(float2 (&v)[16], const float4* twc) {
#pragma unroll
    for (int b0 = 1; b0 < 16; b0 += 4) {
#pragma unroll
        for (int b = b0; b < b0 + 4 && b < 16; ++b) v[b] = tmul<(SG > 0)>(v[b], twc[b * L]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ------------------------------------------------------------ line transforms
// Each line owns its exchange slots (l * SL .. l * SL + 15 * SB + L - 1, below
// (l + 1) * SL).  Where the lanes of a line sit in one wave (GEO::WAVE_LOCAL:
// thread = line * L + lane, 64 / L lines per wave) an exchange only orders the
// wave's own LDS accesses and needs no workgroup barrier: LDS operations of one
// wave execute in issue order, and the fences keep the compiler from moving
// accesses across the exchange.  Code that next touches the buffer with a
// workgroup-wide pattern (relayout, reductions) starts with a barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <class GEO> __device__ __forceinline__ void exchange_sync() {
    if constexpr (GEO::WAVE_LOCAL) wave_sync();
    else __syncthreads();
}

// ------------------------------------------------------------ cross-lane exchange
// One butterfly stage of the block transpose: for the register pair
// (x = v[a], y = v[a + 2^j]) the lanes whose lane-in-line index c has bit j
// clear ("lower") hand y to, and take x from, the lanes with bit j set that
// sit D = (64 / L) 2^j wave lanes higher: lower.y <-> upper.x.
template <int D> __device__ __forceinline__ void xstage(float& x, float& y) {
    if constexpr (D == 32) {
        // swaps lanes 32-63 of the first operand with lanes 0-31 of the second
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        x = __uint_as_float(r[0]);
        y = __uint_as_float(r[1]);
    } else if constexpr (D == 16) {
        // swaps the odd 16-lane rows of the first operand with the even rows of the second
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        x = __uint_as_float(r[0]);
        y = __uint_as_float(r[1]);
    } else {
        static_assert(D == 8, "lane distance 8, 16 or 32");
        // rotation by 8 within each 16-lane row (row_ror:8, control 0x128);
        // bank mask 0x3 writes lanes 0-7 of each row (lower), 0xC lanes 8-15
        const int xi = __float_as_int(x), yi = __float_as_int(y);
        const int yn = __builtin_amdgcn_update_dpp(yi, xi, 0x128, 0xF, 0x3, false);
        const int xn = __builtin_amdgcn_update_dpp(xi, yi, 0x128, 0xF, 0xC, false);
        x = __int_as_float(xn);
        y = __int_as_float(yn);
    }
}

// Transpose, in every line, each L x L block of registers against the line's
// L lanes (register B0 + a of lane c <-> register B0 + c of lane a): one
// stage per bit of the lane index, lanes placed as in line_of.
template <int L> __device__ __forceinline__ void xlane_transpose(float2 (&v)[16]) {
    constexpr int LPW = 64 / L;
#pragma unroll
    for (int j = 0; (1 << j) < L; ++j) {
        const int e = 1 << j;
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            if (a & e) continue;
            switch (LPW * e) {
                case 8: xstage<8>(v[a].x, v[a + e].x); xstage<8>(v[a].y, v[a + e].y); break;
                case 16: xstage<16>(v[a].x, v[a + e].x); xstage<16>(v[a].y, v[a + e].y); break;
                default: xstage<32>(v[a].x, v[a + e].x); xstage<32>(v[a].y, v[a + e].y); break;
            }
        }
    }
}

// NAT -> MID, DFT of sign SG along every line.
// With HALF the exchange runs in two rounds through the slots of b < 8: the
// first moves registers 0..7 (read back by the blocks be < G/2, whose
// sources b = c + L*be are < 8), the second registers 8..15.
template <class GEO, int SG>
__device__ __forceinline__ void nat2mid(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    constexpr int L = GEO::L, G = 16 / L;
    constexpr int R = HalfX<GEO>::value ? 2 : 1;      // rounds
    dft16<SG>(v);
    twiddle_pass<L, SG>(v, tw + c);
    if constexpr (XLaneX<GEO>::value) {
        xlane_transpose<L>(v);
#pragma unroll
        for (int be = 0; be < G; ++be) dftL<L, SG>(&v[be * L]);
        return;
    }
#pragma unroll
    for (int h = 0; h < R; ++h) {
        constexpr int NB = 16 / R, NBE = G / R;
#pragma unroll
        for (int b = 0; b < NB; ++b) lds[slot_x<GEO>(l, b, c)] = v[h * NB + b];
        exchange_sync<GEO>();
#pragma unroll
        for (int be = 0; be < NBE; ++be)
#pragma unroll
            for (int a = 0; a < L; ++a) v[(h * NBE + be) * L + a] = lds[slot_x<GEO>(l, c + L * be, a)];
        exchange_sync<GEO>();
    }
#pragma unroll
    for (int be = 0; be < G; ++be) dftL<L, SG>(&v[be * L]);
}

// MID -> NAT, DFT of sign SG along every line.
template <class GEO, int SG>
__device__ __forceinline__ void mid2nat(float2 (&v)[16], float2* lds, const float4* tw, int l, int c) {
    constexpr int L = GEO::L, G = 16 / L;
    constexpr int R = HalfX<GEO>::value ? 2 : 1;      // rounds, as in nat2mid
#pragma unroll
    for (int be = 0; be < G; ++be) dftL<L, SG>(&v[be * L]);
    if constexpr (XLaneX<GEO>::value) {
        xlane_transpose<L>(v);
        twiddle_pass<L, SG>(v, tw + c);
        dft16<SG>(v);
        return;
    }
#pragma unroll
    for (int h = 0; h < R; ++h) {
        constexpr int NB = 16 / R, NBE = G / R;
#pragma unroll
        for (int be = 0; be < NBE; ++be)
#pragma unroll
            for (int a = 0; a < L; ++a) lds[slot_x<GEO>(l, c + L * be, a)] = v[(h * NBE + be) * L + a];
        exchange_sync<GEO>();
#pragma unroll
        for (int b = 0; b < NB; ++b) v[h * NB + b] = lds[slot_x<GEO>(l, b, c)];
        exchange_sync<GEO>();
    }
    twiddle_pass<L, SG>(v, tw + c);
    dft16<SG>(v);
}

// Re-distribute the field from layout (D0, K0) to (D1, K1) through LDS.
template <int N, int D0, int K0, int D1, int K1>
__device__ __forceinline__ void relayout(float2 (&v)[16], float2* lds, int l, int c) {
    __syncthreads();            // other waves may still read their line-exchange slots
    if constexpr (WaveGeo<N>::HALF) {
        // real parts, then imaginary parts: until its own imaginary parts are
        // written a thread's .y registers still hold the old layout
        float* f = reinterpret_cast<float*>(lds);
        constexpr int SYF = WaveGeo<N>::SYF;
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int y, x;
                reg_yx<N, D0, K0>(l, c, r, y, x);
                f[y * SYF + x] = part ? v[r].y : v[r].x;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int y, x;
                reg_yx<N, D1, K1>(l, c, r, y, x);
                (part ? v[r].y : v[r].x) = f[y * SYF + x];
            }
            __syncthreads();
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, D0, K0>(l, c, r, y, x);
        lds[slot_t<N>(y, x)] = v[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int y, x;
        reg_yx<N, D1, K1>(l, c, r, y, x);
        v[r] = lds[slot_t<N>(y, x)];
    }
    __syncthreads();
}

// fftfreq index -> signed frequency in cycles per pixel times N
template <int N> __device__ __forceinline__ int sfreq(int n) { return n < N / 2 ? n : n - N; }

// XCD-aware block order: the hardware deals consecutive workgroups round
// robin over 8 XCDs (each with its own L2); renumber so that each XCD gets a
// contiguous range of logical ids (neighbouring positions / modes share L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int q = nb / 8, r = nb % 8;
    int x = b % 8;
    return x * q + min(x, r) + b / 8;
}

}  // namespace ptyr
