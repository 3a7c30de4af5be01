// Domain selection (paper Sec. III-B): persistent, replica-parallel engine.
//
// Replicas are independent trajectories, so a workgroup owns RG replicas and
// all n spins of them for the whole run: no workgroup ever waits for another.
// Angles, ADAM moments and (when they fit) sin/cos of the angles live in
// registers for all steps; the current vertex lives in LDS, double-buffered,
// as one bit per (spin, replica) packed into one word per spin.  A step is
//
//   y   = J s                 coupling product, gathered from LDS
//   E  += s (y + h)           energy of the current vertex (wavefront shuffles,
//                             then one fixed-order sum over wavefronts)
//   t   = y - mu s + h;  g = cos(theta) t;  L += sin(theta) t
//   theta <- GD / ADAM update, wrapped to [-pi, pi] with a two-constant 2 pi
//   s'  = sgn(sin theta)      next vertex, written to the other LDS buffer
//
// with one workgroup barrier per step.  The best-vertex bookkeeping is
// pipelined: wavefront 0 compares E_t with the best energy after the barrier of
// step t and publishes a bit per replica; every thread applies it after the
// barrier of step t+1, copying its bits of s_t (still held in registers).
//
// Coupling formats:
//   CK_PM    all couplings +-w: entries col | (J<0) << 31.  The product counts,
//            per replica, the neighbours with J_ij s_j = -w by adding
//            (bit_j xor sign_ij) in packed lanes; y = w (deg - 2 count), exact.
//   CK_PMS   the same couplings staged in LDS for the whole run.  The vertex
//            buffer holds each word twice, as is and complemented per
//            replica, so a neighbour with J < 0 reads the complement and every
//            neighbour costs one LDS read and one packed add:
//            count = sum_j word_j(sign).  Rows are placed on threads in order of
//            decreasing degree, so the 64 rows of a wavefront have nearly equal
//            degree and share one loop count; a wavefront's entries are stored
//            group-major (group k of its 64 lanes contiguous), and each row's
//            neighbours are ordered so that at every read the lanes of a
//            wavefront tend to hit distinct LDS banks.
//   CK_PME   +-w couplings of degree <= 4 with one replica per workgroup: 8 or more
//            spins per thread on 768-1024 threads for large problems, 4 or 8 on 256
//            threads for n <= 2048; fixed-width rows in global memory, a spin's four
//            entries 2 col + (J < 0) in one 16-byte word loaded a few spins ahead
//            (kept in registers for the whole run in the small form), into a vertex
//            buffer holding each spin's byte and its complement; the field (FP32,
//            per position) loaded with the rows.
//   CK_CSRV  CSR values in the state precision.
//   CK_DENSE dense rows in the state precision (small problems).
#include "internal.hpp"

#include <cmath>

namespace ising {

namespace {

template <int RG>
struct SpinWord;
template <>
struct SpinWord<1> {
    using T = uint8_t;
    static constexpr uint32_t ones = 0x1u;
    static constexpr int width = 32;
    __device__ static constexpr int shift(int) { return 0; }
};
template <>
struct SpinWord<2> {
    using T = uint32_t;
    static constexpr uint32_t ones = 0x00010001u;
    static constexpr int width = 16;
    __device__ static constexpr int shift(int r) { return 16 * r; }
};
template <>
struct SpinWord<4> {
    using T = uint32_t;
    static constexpr uint32_t ones = 0x01010101u;
    static constexpr int width = 8;
    __device__ static constexpr int shift(int r) { return 8 * r; }
};

template <typename Real>
struct Consts;
template <>
struct Consts<float> {
    // 2 pi = hi + lo to about 2^-48 relative
    static constexpr float twopi_hi = 6.28318548202514648f;
    static constexpr float twopi_lo = -1.7484555314695172e-07f;
    static constexpr float inv_twopi = 0.159154943091895336f;
};
template <>
struct Consts<double> {
    static constexpr double twopi_hi = 6.283185307179586232;
    static constexpr double twopi_lo = 2.4492935982947064e-16;
    static constexpr double inv_twopi = 0.15915494309189533577;
};

// minimax coefficients (rounded to float) of sin r = r + r^3 (C1 + C2 z + C3 z^2) and
// cos r = 1 + z (C1 + C2 z + C3 z^2 + C4 z^3), z = r^2, |r| <= pi/4
constexpr float SIN_C1 = -1.666666716e-01f, SIN_C2 = 8.332728408e-03f, SIN_C3 = -1.957433851e-04f;
constexpr float COS_C1 = -5.000000000e-01f, COS_C2 = 4.166666791e-02f, COS_C3 = -1.388838165e-03f, COS_C4 = 2.455472713e-05f;

// sin and cos of |x| <= 5 pi / 4 in float (angles here are wrapped to [-pi, pi]):
// quadrant k = rint(x 2/pi) in {-2, ..., 2}, reduction r = x - k pi/2 with pi/2 split
// in three parts (each step one FMA, Cody-Waite style), polynomials in z = r^2 on
// |r| <= pi/4 whose coefficients minimise the maximum error of sin (relative) and
// cos (absolute) over that interval (about 9e-9 and 1e-9, below float rounding),
// then the rotation by k pi/2: cos(k pi/2) = 1 - |k| and sin(k pi/2) = k (2 - |k|)
// for |k| <= 2, so both results are one exact product plus one FMA.
__device__ inline void dsincos(float x, float *s, float *c) {
    const float k = rintf(x * 0.636619772367581343f);
    float r = __builtin_fmaf(-k, 1.57079637050628662f, x);
    r = __builtin_fmaf(-k, -4.37113882867379300e-08f, r);
    r = __builtin_fmaf(-k, -1.71512451000588190e-15f, r);
    const float z = r * r;
    float ps = __builtin_fmaf(z, SIN_C3, SIN_C2);
    ps = __builtin_fmaf(z, ps, SIN_C1);
    const float sn = __builtin_fmaf(r * z, ps, r);
    float pc = __builtin_fmaf(z, COS_C4, COS_C3);
    pc = __builtin_fmaf(z, pc, COS_C2);
    pc = __builtin_fmaf(z, pc, COS_C1);
    const float cn = __builtin_fmaf(z, pc, 1.0f);
    const float ck = 1.0f - __builtin_fabsf(k);
    const float sk = k * (2.0f - __builtin_fabsf(k));
    *s = __builtin_fmaf(sk, cn, ck * sn);
    *c = __builtin_fmaf(-sk, sn, ck * cn);
}
__device__ inline void dsincos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ inline float dsin(float x) {
    float s, c;
    dsincos(x, &s, &c);
    return s;
}
__device__ inline double dsin(double x) { return sin(x); }
// dsin(x) < 0 from the range reduction alone: in the odd quadrants the sine is +-cos(r)
// (|r| <= pi/4, never zero), in the even ones +-sin(r), whose polynomial keeps the sign of r
// (the rotation by k keeps or flips it).  The same decision as dsin(x) < 0 for |x| <= 4.
__device__ inline bool dsin_neg(float x) {
    const float k = rintf(x * 0.636619772367581343f);
    float r = __builtin_fmaf(-k, 1.57079637050628662f, x);
    r = __builtin_fmaf(-k, -4.37113882867379300e-08f, r);
    r = __builtin_fmaf(-k, -1.71512451000588190e-15f, r);
    const int q = (int)k & 3;
    return q == 3 || (q == 0 && r < 0.f) || (q == 2 && r > 0.f);
}
__device__ inline bool dsin_neg(double x) { return sin(x) < 0; }
// sin(x) < 0 for |x| <= 4, which holds for every angle the step has wrapped (|x| exceeds pi by at
// most a rounding error): the sign of x, flipped where |x| is at least the float just above pi.
// Checked against the sign of the float64 sine for every float in [-4, 4]; dsin_neg takes the
// same decision there, in 11 instructions instead of 2.
__device__ inline bool wrapped_sin_neg(float x) { return (x < 0.f) != (__builtin_fabsf(x) >= 3.14159274f); }
__device__ inline bool wrapped_sin_neg(double x) { return dsin_neg(x); }
// cos x for a wrapped angle (|x| exceeds pi by at most a rounding error): cos x = -sin f with
// f = |x| - pi/2 in [-pi/2, pi/2] (pi/2 in two parts), and sin f = f + f^3 (S1 + S2 z + S3 z^2 + S4 z^3),
// z = f^2, coefficients (rounded to float) fitted to the relative error of sin on [0, pi/2] by
// iteratively reweighted least squares (Lawson's algorithm): 6e-9, below float rounding.  Eight
// instructions; a float emulation over 2e7 random angles and 2e6 around 0, +-pi/2 and +-pi gives
// at most 1.8 ulp.
constexpr float WCOS_S1 = -1.6666660e-01f, WCOS_S2 = 8.3330665e-03f, WCOS_S3 = -1.9809604e-04f,
                WCOS_S4 = 2.6057808e-06f;
__device__ inline float wrapped_cos(float x) {
    const float f = (__builtin_fabsf(x) - 1.57079637050628662f) - -4.37113882867379300e-08f;
    const float z = f * f;
    float p = __builtin_fmaf(z, WCOS_S4, WCOS_S3);
    p = __builtin_fmaf(z, p, WCOS_S2);
    p = __builtin_fmaf(z, p, WCOS_S1);
    return __builtin_fmaf(-f * z, p, -f);
}
__device__ inline double wrapped_cos(double x) { return cos(x); }
__device__ inline float dasin(float x) { return asinf(x); }
__device__ inline double dasin(double x) { return asin(x); }
// a word in global memory, addressed as such (an address made opaque to the compiler would
// otherwise be read with flat loads, which a wait for LDS reads also waits for)
using GlobalU32 = __attribute__((address_space(1))) uint32_t;
using U32x4 = uint32_t __attribute__((ext_vector_type(4)));
using GlobalU32x4 = __attribute__((address_space(1))) U32x4;
using GlobalF32 = __attribute__((address_space(1))) float;
using LdsU8 = __attribute__((address_space(3))) uint8_t;
using LdsI8 = __attribute__((address_space(3))) const int8_t;
using LdsU16 = __attribute__((address_space(3))) uint16_t;
// Bytes per parity of the fixed-width-row form's vertex buffer: a signed byte per position and
// copy (+-1 and its negation) for ept * block positions and the zero pair, rounded to 16.
__host__ __device__ constexpr int twin_stride(int ept, int block) { return (2 * (ept * block + 1) + 15) / 16 * 16; }
// The fixed-width-row form's vertex buffers: a static LDS array per kernel.  Its address is fixed
// when the kernel is compiled, so a read at (row entry + parity offset) or (own position + offset)
// carries the constant part as the instruction's immediate offset instead of an add per access.
template <int BYTES>
__device__ __forceinline__ unsigned char *twin_lds() {
    __shared__ __align__(16) unsigned char buf[BYTES];
    return buf;
}
// a compile-time flag passed to a generic lambda
template <bool B>
struct Flag {
    static constexpr bool value = B;
};
// a compile-time integer passed to a generic lambda
template <int V>
struct IntC {
    static constexpr int value = V;
};

// fused multiply-add in the state precision (the plain builtin takes and returns double)
__device__ inline float dfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double dfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float dsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float drint(float x) { return rintf(x); }
__device__ inline float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double drcp(double x) { return 1.0 / x; }

__device__ inline double drint(double x) { return rint(x); }

// One GD or ADAM step of an angle, wrapped to [-pi, pi] with the two-constant 2 pi: the same
// operations in every engine form, with contraction off so that only the written FMAs fuse.
template <typename Real>
__device__ __forceinline__ Real angle_step(Real th, Real &mo, Real &ve, Real g, bool adam, Real b1, Real omb1,
                                           Real b2, Real omb2, Real lib1, Real lr, Real ib2, Real eps) {
#pragma clang fp contract(off)
    Real upd;
    if (adam) {
        mo = dfma(b1, mo, omb1 * g);
        ve = dfma(b2, ve, omb2 * (g * g));
        upd = (mo * lib1) * drcp(dsqrt(ve * ib2) + eps);
    } else {
        upd = lr * g;
    }
    Real tn = th - upd;
    const Real q = drint(tn * Consts<Real>::inv_twopi);
    tn = dfma(-q, Consts<Real>::twopi_hi, tn);
    return dfma(-q, Consts<Real>::twopi_lo, tn);
}

// The same step for the fixed-width-row form, with the moments kept scaled in registers,
// mo = m / (1 - b1) and ve = v / (1 - b2), so that each moment update is one FMA:
// m' = b1 m + (1 - b1) g  <=>  mo' = b1 mo + g, and likewise for v with g^2; the update
// lr m_hat / (sqrt(v_hat) + eps) is then (mo a1) / (sqrt(ve a2) + eps) with a1 = lr (1 - b1) / (1 - b1^t)
// and a2 = (1 - b2) / (1 - b2^t) per step.  The moments are scaled when they are read and unscaled
// when they are written back, so the state holds m and v as in every other form.  The angle is
// returned unwrapped: wrap_angle below is the wrap.
template <typename Real>
__device__ __forceinline__ Real angle_step_scaled(Real th, Real &mo, Real &ve, Real g, bool adam, Real b1, Real b2,
                                                  Real a1, Real lr, Real a2, Real eps) {
#pragma clang fp contract(off)
    Real upd;
    if (adam) {
        if constexpr (sizeof(Real) == 4) {
            // mo = mo b1 + g and ve = ve b2 + g^2, each written in place (the compiler's accumulate
            // form would write into g's register and copy back: two moves per update)
            const Real g2 = g * g;
            asm("v_fma_f32 %0, %0, %1, %2" : "+v"(mo) : "v"(b1), "v"(g));
            asm("v_fma_f32 %0, %0, %1, %2" : "+v"(ve) : "v"(b2), "v"(g2));
        } else {
            mo = dfma(b1, mo, g);
            ve = dfma(b2, ve, g * g);
        }
        // th - a1 mo / (sqrt(ve a2) + eps), the last product and the difference in one FMA
        const Real q = mo * drcp(dsqrt(ve * a2) + eps);
        return dfma(-q, a1, th);
    }
    return dfma(-g, lr, th);
}

// theta - 2 pi rint(theta / 2 pi) with 2 pi in two parts; the identity for |theta| < 3, where the
// quotient rounds to 0
template <typename Real>
__device__ __forceinline__ Real wrap_angle(Real tn) {
    const Real q = drint(tn * Consts<Real>::inv_twopi);
    tn = dfma(-q, Consts<Real>::twopi_hi, tn);
    return dfma(-q, Consts<Real>::twopi_lo, tn);
}

// Output number (c + 1) of SplitMix64 seeded with `seed` (Steele, Lea, Flood 2014).
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// U = 2 * top24 / 2^24 - 1, exact in float and double
template <typename Real>
__device__ inline Real draw_uniform(uint64_t seed, int r, int i) {
    const uint64_t z = splitmix64(seed, ((uint64_t)(uint32_t)r << 32) | (uint32_t)i);
    const Real u24 = (Real)(uint32_t)(z >> 40);
    return (Real)2 * (u24 * (Real)5.9604644775390625e-08) - (Real)1;
}

// Sum over the 64 lanes of a wavefront in a fixed order, result in every lane.
// float: DPP adds within quads, half-rows and rows, then the row broadcasts of
// lane 15 and lane 31 accumulate the four rows into lane 63, which is read back.
// double: butterfly of lane shuffles.
__device__ inline float wave_sum(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// The staged-image engine with the relaxed-vertex loss is its own instantiation
// (template coupling CK_PMSR), so that the vertex-loss one carries none of its registers.
constexpr int CK_PMSR = 4;
__host__ __device__ constexpr bool is_pms(int ck) { return ck == CK_PMS || ck == CK_PMSR; }
// The wide packed engine with fixed-width neighbour rows (DSArgs::ell) is its own
// instantiation too (template coupling CK_PME), with no CSR path in its step.
constexpr int CK_PME = 5;

template <typename Real, int CK, int RG>
__device__ inline void coupling(const DSArgs &a, int i, const typename SpinWord<RG>::T *sc, Real (&y)[RG],
                                const uint2 *img = nullptr, int g0 = 0, uint32_t cnt = 0) {
    using SW = SpinWord<RG>;
    if constexpr (is_pms(CK)) {
        using T = typename SW::T;
        const unsigned char *sb = (const unsigned char *)sc;
        // every lane of a wavefront has the same group count
        const int G = __builtin_amdgcn_readfirstlane((int)(cnt >> 16));
        const uint2 *q = img + g0;
        uint32_t acc = 0;
        for (int k = 0; k < G; ++k) {
            const uint2 v = q[64 * k];
            acc += (uint32_t)(*(const T *)(sb + (v.x & 0xffffu))) + (uint32_t)(*(const T *)(sb + (v.x >> 16))) +
                   (uint32_t)(*(const T *)(sb + (v.y & 0xffffu))) + (uint32_t)(*(const T *)(sb + (v.y >> 16)));
        }
        const int deg = (int)(cnt & 0xffffu);
        const Real w = (Real)a.w;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const uint32_t c = SW::width == 32 ? acc : ((acc >> SW::shift(r)) & ((1u << SW::width) - 1u));
            y[r] = w * (Real)(deg - 2 * (int)c);
        }
    } else if constexpr (CK == CK_PM) {
        const int rs = a.row_ptr[i], re = a.row_ptr[i + 1];
        uint32_t acc = 0;
        for (int q = rs; q < re; ++q) {
            const uint32_t e = a.pm[q];
            const uint32_t nm = (uint32_t)((int32_t)e >> 31) & SW::ones;
            acc += (uint32_t)sc[e & 0x7fffffffu] ^ nm;
        }
        const int deg = re - rs;
        const Real w = (Real)a.w;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const uint32_t cnt = SW::width == 32 ? acc : ((acc >> SW::shift(r)) & ((1u << SW::width) - 1u));
            y[r] = w * (Real)(deg - 2 * (int)cnt);
        }
    } else {
#pragma unroll
        for (int r = 0; r < RG; ++r) y[r] = 0;
        if constexpr (CK == CK_CSRV) {
            const Real *val = (const Real *)a.val;
            const int rs = a.row_ptr[i], re = a.row_ptr[i + 1];
            for (int q = rs; q < re; ++q) {
                const Real v = val[q];
                const uint32_t wd = (uint32_t)sc[a.col[q]];
#pragma unroll
                for (int r = 0; r < RG; ++r) y[r] += ((wd >> SW::shift(r)) & 1u) ? -v : v;
            }
        } else {
            const Real *row = (const Real *)a.J + (size_t)i * a.n;
            for (int j = 0; j < a.n; ++j) {
                const Real v = row[j];
                const uint32_t wd = (uint32_t)sc[j];
#pragma unroll
                for (int r = 0; r < RG; ++r) y[r] += ((wd >> SW::shift(r)) & 1u) ? -v : v;
            }
        }
    }
}

// z = J x for the relaxed-vertex loss, x = sin(theta) staged in LDS as [spin][RG]
// (CSR in row order, dense rows in column order).  CK_PMS: the staged image's entries
// address x and its negation, laid out like the vertex words and their complements
// (record of position q at XS times the word's byte offset), so each neighbour is one
// LDS read of RG values and RG adds, in the image's order, then the common magnitude.
template <typename Real, int RG>
struct XRec {
    Real v[RG];
};
template <typename Real, int CK, int RG>
__device__ inline void relaxed_product(const DSArgs &a, int i, const Real *xc, Real (&z)[RG],
                                       const uint2 *img = nullptr, int g0 = 0, uint32_t cnt = 0) {
#pragma unroll
    for (int r = 0; r < RG; ++r) z[r] = 0;
    if constexpr (is_pms(CK)) {
        constexpr int XS = RG * (int)sizeof(Real) / (int)sizeof(typename SpinWord<RG>::T);
        const unsigned char *xb = (const unsigned char *)xc;
        const int G = __builtin_amdgcn_readfirstlane((int)(cnt >> 16));
        const uint2 *q = img + g0;
        for (int k = 0; k < G; ++k) {
            const uint2 v = q[64 * k];
            const uint32_t e[4] = {v.x & 0xffffu, v.x >> 16, v.y & 0xffffu, v.y >> 16};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const XRec<Real, RG> x = *(const XRec<Real, RG> *)(xb + (size_t)XS * e[h]);
#pragma unroll
                for (int r = 0; r < RG; ++r) z[r] += x.v[r];
            }
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) z[r] *= (Real)a.w;
    } else if constexpr (CK == CK_PM) {
        const int rs = a.row_ptr[i], re = a.row_ptr[i + 1];
        for (int q = rs; q < re; ++q) {
            const uint32_t e = a.pm[q];
            const Real sg = (e >> 31) ? (Real)-1 : (Real)1;
            const Real *xj = xc + (size_t)(e & 0x7fffffffu) * RG;
#pragma unroll
            for (int r = 0; r < RG; ++r) z[r] = dfma(sg, xj[r], z[r]);
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) z[r] *= (Real)a.w;
    } else if constexpr (CK == CK_CSRV) {
        const Real *val = (const Real *)a.val;
        const int rs = a.row_ptr[i], re = a.row_ptr[i + 1];
        for (int q = rs; q < re; ++q) {
            const Real v = val[q];
            const Real *xj = xc + (size_t)a.col[q] * RG;
#pragma unroll
            for (int r = 0; r < RG; ++r) z[r] = dfma(v, xj[r], z[r]);
        }
    } else if constexpr (CK == CK_DENSE) {
        const Real *row = (const Real *)a.J + (size_t)i * a.n;
        for (int j = 0; j < a.n; ++j) {
            const Real v = row[j];
#pragma unroll
            for (int r = 0; r < RG; ++r) z[r] = dfma(v, xc[(size_t)j * RG + r], z[r]);
        }
    }
}

// 28 or 32 spins per thread (one replica per workgroup, large n) keep 84 or 96 state registers
// per thread: at most 768 threads, so that the register budget is 168
constexpr int launch_bound(int ept) { return ept >= 28 ? 768 : 1024; }

// With 8 or more spins per thread the per-spin loads (row bounds, field) and the write-back
// addresses would be hoisted out of the step loop and kept live for every spin, which
// exceeds the register budget; an opaque copy of the spin index (an empty asm on a
// register, no memory access) makes them local to each use.
template <int EPT>
__device__ __forceinline__ int local_index(int i) {
    if constexpr (EPT >= 8) asm volatile("" : "+v"(i));
    return i;
}

// OPT: the optimizer as a compile-time choice (0 GD, 1 ADAM) or -1 to read it at run time.
// LOSS (fixed-width-row form only): false for runs that need no loss (no loss trace and no
// convergence test), whose update then evaluates cos(theta) alone and takes the vertex sign
// from the bit it already holds; true computes sin(theta) as well, for the loss.  Both run
// the same update of the angles, so their trajectories are identical.
// PLAIN (fixed-width-row form without the loss only): unit couplings (w = 1) and no field, so the
// product is the integer sum itself and no per-position field is loaded; the same results as
// the general form (y = fma(1, sum, 0) = sum exactly).
// LBX (fixed-width-row form only): the workgroup size when it is not launch_bound(EPT): small
// problems run one replica per workgroup of kPmeSmallBlock threads (pme_small_ept spins each),
// whose few records and fields per thread stay in registers for the whole run.
template <typename Real, int CK, int RG, int EPT, int OPT = -1, bool LOSS = true, bool PLAIN = false, int LBX = 0>
__device__ __forceinline__ void ds_body(const DSArgs &a, const int r0) {
    using SWd = SpinWord<RG>;
    using SW = typename SWd::T;
    constexpr int NE = EPT * RG;
    // keep sin/cos of theta in registers (not in the fixed-width-row form, which evaluates
    // cos(theta) once per update)
    constexpr bool KEEP = NE * (int)sizeof(Real) <= 32 && CK != CK_PME;
    static_assert(NE <= 32, "one 32-bit mask per thread");
    extern __shared__ __align__(16) unsigned char smem[];

    const int n = a.n, B = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, NW = B >> 6;
    // Vertex buffers, double-buffered by step parity.  CK_PMS: each parity holds
    // a region of words (position q of the thread layout) and a region of their
    // per-replica complements, a.pms_rb bytes each, with a zero word at position
    // EPT*B for padded slots.  CK_PME: per parity (TWS bytes), each spin's sign s as a signed
    // byte and its negation side by side (bytes 2 i, 2 i + 1), so that a row entry
    // 2 col + (J < 0) reads the neighbour's term sgn(J) s_col directly; the pair at position
    // EPT LB is kept zero for unused entries.  Other couplings: npad words per parity, indexed by
    // spin, word n kept zero.
    constexpr bool TWIN = CK == CK_PME;
    // The fixed-width-row form runs with B = launch_bound(EPT) (checked at launch), so its
    // positions e LB + tid and the parity stride of its vertex buffer are compile-time constants
    // and its LDS reads and writes take them as immediate offsets.
    constexpr int LB = LBX > 0 ? LBX : launch_bound(EPT);
    constexpr int TWS = twin_stride(EPT, LB);
    const int npad = EPT * B + 1;
    // (the fixed-width-row form's vertex buffers are static, outside the dynamic LDS)
    const size_t vbytes = is_pms(CK) ? (size_t)4 * a.pms_rb : TWIN ? 0 : (size_t)2 * npad * sizeof(SW);
    SW *sbuf = (SW *)smem;
    const size_t off = (vbytes + 15) & ~(size_t)15;
    Real *ep = (Real *)(smem + off);      // [2][NW][RG]
    Real *lp = ep + 2 * NW * RG;          // [2][NW][RG]
    uint32_t *flg = (uint32_t *)(lp + 2 * NW * RG);  // [2]
    uint2 *img = (uint2 *)(smem + ((off + 2 * 2 * NW * RG * sizeof(Real) + 8 + 15) & ~(size_t)15));
    // relaxed-vertex loss: sin(theta) per parity.  Other couplings: [npad][RG] where the image
    // would be.  CK_PMS: after the image, per parity a region of records [RG] at XS times the
    // vertex word's byte offset (XS * a.pms_rb bytes) and a region of their negations.
    constexpr bool CAN_RELAX = CK != CK_PMS && CK != CK_PME;  // the fixed-width rows serve the vertex loss only
    constexpr int XS = RG * (int)sizeof(Real) / (int)sizeof(SW);
    const bool relaxed = CK == CK_PMSR || (CK != CK_PMS && a.loss == ISING_LOSS_RELAXED);
    const size_t img_off = (size_t)((unsigned char *)img - smem);
    const size_t x_off = is_pms(CK) ? ((img_off + (size_t)8 * a.pimg_groups + 15) & ~(size_t)15) : img_off;
    Real *xb = (Real *)(smem + x_off);
    const size_t xpar = is_pms(CK) ? (size_t)2 * XS * a.pms_rb : (size_t)npad * RG * sizeof(Real);  // bytes per parity
    // convergence test: per wavefront, the window of losses [kConvWindowMax][RG] and L_1 [RG]
    // (the fixed-width-row form without the loss runs neither the test nor a loss trace; its
    // launch checks that)
    constexpr bool NOLOSS = CK == CK_PME && !LOSS;
    const bool conv = !NOLOSS && a.conv_tol > 0;
    const size_t tail = relaxed ? x_off + 2 * xpar : (is_pms(CK) ? img_off + (size_t)8 * a.pimg_groups : img_off);
    Real *cring = (Real *)(smem + ((tail + 15) & ~(size_t)15)) + (size_t)wave * (kConvWindowMax + 1) * RG;
    int prow_r[is_pms(CK) ? EPT : 1];
    uint32_t pcnt_r[is_pms(CK) ? EPT : 1];
    int row_r[is_pms(CK) ? EPT : 1];  // spin held at position e * B + tid
    if constexpr (is_pms(CK)) {
        const uint2 *src = (const uint2 *)a.pimg;
        for (int q = tid; q < a.pimg_groups; q += B) img[q] = src[q];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int q = e * B + tid;
            prow_r[e] = a.prow[q];
            pcnt_r[e] = a.pcnt[q];
            row_r[e] = q < n ? a.pperm[q] : 0;
        }
    }
    auto spin_of = [&](int e) -> int {
        if constexpr (is_pms(CK)) return row_r[e];
        else return e * B + tid;
    };
    // Fixed-width-row form: twb, the LDS address of its buffers (parity par at twb + par TWS);
    // tw0, tw1 the lane's own pair (2 tid) from twb and from twb + 32768, kept opaque so that
    // each access to position e takes the base whose immediate offset stays below 2^16.
    uint32_t twb = 0, tw0 = 0, tw1 = 0;
    if constexpr (TWIN) {
        twb = (uint32_t)(size_t)(LdsU8 *)twin_lds<2 * TWS>();
        tw0 = twb + 2 * tid;
        tw1 = tw0 + 32768;
        asm volatile("" : "+v"(tw0), "+v"(tw1));
    }
    // the lane's pair of position e in parity par (compile-time constants in the step, where the
    // choice of base folds away; either base gives the same address)
    auto tw_pos = [&](int par, int e) -> uint32_t {
        const int off = par * TWS + 2 * e * LB;
        return off < 65536 ? tw0 + off : tw1 + (off - 32768);
    };
    // vertex buffer of parity par, as the coupling reads it
    auto vbuf = [&](int par) -> SW * {
        if constexpr (is_pms(CK)) return (SW *)(smem + (size_t)par * 2 * a.pms_rb);
        else if constexpr (TWIN) return (SW *)nullptr;  // addressed through tw_pos and twb
        else return sbuf + par * npad;
    };
    auto put = [&](int par, int e, SW word) {
        SW *S = vbuf(par);
        if constexpr (is_pms(CK)) {
            S[e * B + tid] = word;
            ((SW *)((unsigned char *)S + a.pms_rb))[e * B + tid] = (SW)(word ^ (SW)SWd::ones);
        } else if constexpr (TWIN) {
            static_assert(sizeof(SW) == 1, "one byte per spin and copy");
            (void)S;
            // word 1 (s = -1): bytes -1, +1; word 0 (s = +1): bytes +1, -1
            *(LdsU16 *)(size_t)tw_pos(par, e) = word ? (uint16_t)0x01FFu : (uint16_t)0xFF01u;
        } else {
            S[e * B + tid] = word;
        }
    };
    // sin(theta) of position q, replica r, for the step of parity par (and its negation for CK_PMS)
    auto putx = [&](int par, int q, int r, Real v) {
        unsigned char *xp = (unsigned char *)xb + (size_t)par * xpar;
        if constexpr (is_pms(CK)) {
            ((Real *)(xp + (size_t)q * RG * sizeof(Real)))[r] = v;
            ((Real *)(xp + (size_t)XS * a.pms_rb + (size_t)q * RG * sizeof(Real)))[r] = -v;
        } else {
            ((Real *)xp)[(size_t)q * RG + r] = v;
        }
    };
    if (is_pms(CK) && relaxed && tid < RG)  // the padded slot reads zero records
        for (int par = 0; par < 2; ++par) putx(par, EPT * B, tid, (Real)0);
    if (tid == 0) {
        if constexpr (is_pms(CK)) {
            vbuf(0)[EPT * B] = 0;
            vbuf(1)[EPT * B] = 0;
        } else if constexpr (TWIN) {
            *(LdsU16 *)(size_t)(twb + 2 * EPT * LB) = 0;
            *(LdsU16 *)(size_t)(twb + TWS + 2 * EPT * LB) = 0;
        } else {
            sbuf[n] = 0;
            sbuf[npad + n] = 0;
        }
    }
    const Real *hv = (const Real *)a.h;
    Real *gth = (Real *)a.theta;
    Real *gm = (Real *)a.m;
    Real *gv = (Real *)a.v;
    const bool adam = OPT >= 0 ? OPT == 1 : a.opt == ISING_OPT_ADAM;

    Real th[NE], mo[NE], ve[NE];
    Real xs[KEEP ? NE : 1], cs[KEEP ? NE : 1];
    uint32_t cur = 0, prv = 0, best = 0;

#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int q = e * B + tid;
        const int i = spin_of(e);
        SW word = 0;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const int k = e * RG + r;
            th[k] = 0;
            mo[k] = 0;
            ve[k] = 0;
            if (KEEP) {
                xs[k] = 0;
                cs[k] = 1;
            }
            if (q < n) {
                const size_t idx = (size_t)(r0 + r) * n + i;
                Real t;
                if (a.init_mode == 0) {
                    t = gth[idx];
                    if (t > (Real)3.15 || t < (Real)-3.15) {  // angles the engines write are within pi_f
                        const Real qw = drint(t * Consts<Real>::inv_twopi);
                        t = t - qw * Consts<Real>::twopi_hi;
                        t = t - qw * Consts<Real>::twopi_lo;
                    }
                    if (gm) mo[k] = CK == CK_PME ? gm[idx] / (Real)(1.0 - a.b1) : gm[idx];
                    if (gv) ve[k] = CK == CK_PME ? gv[idx] / (Real)(1.0 - a.b2) : gv[idx];
                    if (a.s_best[idx] < 0) best |= 1u << k;
                } else {
                    const Real u = a.init_mode == 1 ? ((const Real *)a.uniform)[idx]
                                                    : draw_uniform<Real>(a.seed, r0 + r, i);
                    t = dasin(u);
                }
                th[k] = t;
                Real x, c;
                dsincos(t, &x, &c);
                if (KEEP) {
                    xs[k] = x;
                    cs[k] = c;
                }
                if (CAN_RELAX && relaxed) putx(0, q, r, x);
                if (x < 0) {
                    cur |= 1u << k;
                    word |= (SW)(1u << SWd::shift(r));
                }
            }
        }
        if (q < n) put(0, e, word);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (tid < 2) flg[tid] = 0;
    double ebest = INFINITY;
    int bstep = 0;
    // (the fixed-width-row form scores the vertices in every wavefront)
    if ((TWIN || wave == 0) && lane < RG && a.init_mode == 0) {
        ebest = a.e_best[r0 + lane];
        bstep = a.best_step[r0 + lane];
    }
    __syncthreads();

    const Real lr = (Real)a.lr, mu = (Real)a.mu, b1 = (Real)a.b1, b2 = (Real)a.b2, eps = (Real)a.eps;
    const Real omb1 = (Real)(1.0 - a.b1), omb2 = (Real)(1.0 - a.b2);
    const Real *bct = (const Real *)a.bias;  // 1/(1-b1^t), 1/(1-b2^t) for this launch's steps
    const bool trace_l = !NOLOSS && a.ltrace != nullptr;
    uint32_t done = 0;          // replicas that have stopped (identical in every wavefront)
    int conv_t = 0;             // wave 0, lane r < RG: step at which replica r stopped
    int tlast = a.steps;        // last step run
    if (conv && a.t0 > 0) {
        // continuing a run: the replicas that stopped in an earlier call (conv_step > 0) and the
        // window of losses and L_1 carried in conv_state, copied into this wavefront's ring
        uint32_t stopped = 0;
#pragma unroll
        for (int r = 0; r < RG; ++r)
            if (a.conv_step[r0 + r] > 0) stopped |= 1u << r;
        done = (uint32_t)__builtin_amdgcn_readfirstlane((int)stopped);  // uniform: kept in a scalar register
        if (lane < RG) {
            conv_t = a.conv_step[r0 + lane];
            const Real *cs = (const Real *)a.conv_state + (size_t)(r0 + lane) * (kConvWindowMax + 1);
            for (int q = 0; q <= kConvWindowMax; ++q) cring[q * RG + lane] = cs[q];
        }
    }

    // Fixed-width-row form: the vertex is not kept as bits in registers; when a vertex scores
    // best, each lane copies its signs from the parity that holds it (its own positions, which
    // only it writes) before the step that overwrites them.
    bool twimp = false;  // the vertex scored in the last step is the best so far
    auto tw_keep = [&](int par) __attribute__((always_inline)) {
        uint32_t b = 0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) b |= (*(LdsI8 *)(size_t)tw_pos(par, e) < 0 ? 1u : 0u) << e;
        best = b;
    };
    // The small-problem fixed-width-row form (a few spins per thread) keeps its records and fields
    // in registers for the whole run; the large one loads them ahead of each spin in every step.
    constexpr bool ELL_RES = CK == CK_PME && LBX > 0;
    U32x4 nbw_res[ELL_RES ? EPT : 1];
    Real hres[ELL_RES && !PLAIN ? EPT : 1];
    if constexpr (ELL_RES) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            nbw_res[e] = ((const GlobalU32x4 *)((uintptr_t)a.ell + (size_t)e * LB * 16))[tid];
            if constexpr (!PLAIN) hres[e] = ((const GlobalF32 *)((uintptr_t)a.ellh + (size_t)e * LB * 4))[tid];
        }
    }
    // One step t (read parity (t - 1) & 1); returns true when every replica has stopped.
    auto step = [&](auto PC, const int t) __attribute__((always_inline)) -> bool {
        // read parity: compile-time for the fixed-width-row form (RP = 0 at odd t, 1 at even t)
        constexpr int RPc = decltype(PC)::value;
        const int rpar = RPc >= 0 ? RPc : ((t - 1) & 1);
        const SW *sc = vbuf(rpar);
        if constexpr (TWIN) {
            // the vertex scored in the previous step, s^(t-2), is still in the write parity
            if (twimp) tw_keep(1 - RPc);
        }
        const Real ib1 = adam ? bct[2 * (t - 1)] : (Real)1, ib2 = adam ? bct[2 * (t - 1) + 1] : (Real)1;
        const Real lib1 = lr * ib1;
        const Real sa1 = lib1 * omb1, sa2 = ib2 * omb2;  // the scaled-moment form's factors
        Real Ep[RG], Lp[RG];
#pragma unroll
        for (int r = 0; r < RG; ++r) Ep[r] = Lp[r] = (Real)-0.0;  // x + (-0) = x: no add for the first term
        uint32_t nxt = 0;
        // wide packed engine: the fixed-width neighbour words of spin e are loaded ELL_AHEAD
        // spins before its update (the base pointer is opaque per step, so that the loads
        // stay inside the step instead of being hoisted for every spin)
        constexpr bool WIDE_ELL = CK == CK_PME;
        constexpr int ELL_AHEAD = EPT >= 28 ? 2 : 4;  // the widest variants leave little register room
        constexpr bool use_ell = WIDE_ELL && !ELL_RES;
        // a spin's record is contiguous: its four entries in one 16-byte load per lane, coalesced
        // over the wave (every word used: a record with an unused word let that word's register be
        // reused while its load was in flight, which made every spin wait for the load issued
        // ahead of it); the field (or 0) of each position in a separate array, loaded with it
        static_assert(kEllWidth == 4, "one 16-byte record per spin");
        U32x4 nbw[WIDE_ELL ? EPT : 1];
        Real hpre[WIDE_ELL && !PLAIN ? EPT : 1];
        uintptr_t ellp = (uintptr_t)a.ell;
        uintptr_t ellh = (uintptr_t)a.ellh;
        if constexpr (WIDE_ELL) {
            asm volatile("" : "+s"(ellp), "+s"(ellh));
            if (use_ell)
#pragma unroll
                for (int e = 0; e < ELL_AHEAD && e < EPT; ++e) {
                    nbw[e] = ((const GlobalU32x4 *)(ellp + (size_t)e * LB * 16))[tid];
                    if constexpr (!PLAIN) hpre[e] = ((const GlobalF32 *)(ellh + (size_t)e * LB * 4))[tid];
                }
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if constexpr (WIDE_ELL) {
                if (use_ell && e + ELL_AHEAD < EPT) {  // a uniform base per spin plus the lane's offset
                    nbw[e + ELL_AHEAD] = ((const GlobalU32x4 *)(ellp + (size_t)(e + ELL_AHEAD) * LB * 16))[tid];
                    if constexpr (!PLAIN)
                        hpre[e + ELL_AHEAD] = ((const GlobalF32 *)(ellh + (size_t)(e + ELL_AHEAD) * LB * 4))[tid];
                }
            }
            if constexpr (WIDE_ELL) {
                // positions e LB .. e LB + LB - 1: a scalar test first (all in range for every e but
                // the last ones), the per-lane test only where the range ends; the limit is made
                // opaque per step so that the per-lane masks are not all kept across the step loop
                int lim = n - e * LB;
                asm volatile("" : "+s"(lim));
                if (lim < LB && tid >= lim) continue;
            } else {
                if (e * B + tid >= n) continue;
            }
            // (the fixed-width-row form needs no spin index: its rows and vertex are by position)
            const int i = WIDE_ELL ? e * LB + tid : local_index<EPT>(spin_of(e));
            Real y[RG];
            if constexpr (is_pms(CK)) {
                coupling<Real, CK, RG>(a, i, sc, y, img, prow_r[e], pcnt_r[e]);
            } else if constexpr (WIDE_ELL) {
                // one replica per workgroup: the neighbours' terms sgn(J) s as signed bytes, read
                // at immediate offsets of the read parity's buffer; y = w sum + h
                const uint32_t sb = twb + RPc * TWS;
                const U32x4 rec = ELL_RES ? nbw_res[e] : nbw[e];
                const int sum = (int)*(LdsI8 *)(size_t)(sb + rec[0]) + (int)*(LdsI8 *)(size_t)(sb + rec[1]) +
                                (int)*(LdsI8 *)(size_t)(sb + rec[2]) + (int)*(LdsI8 *)(size_t)(sb + rec[3]);
#pragma unroll
                for (int r = 0; r < RG; ++r) {
                    if constexpr (PLAIN) y[r] = (Real)sum;
                    else y[r] = dfma((Real)a.w, (Real)sum, ELL_RES ? hres[e] : hpre[e]);
                }
            } else {
                coupling<Real, CK, RG>(a, i, sc, y);
            }
            Real z[RG];
            if constexpr (CAN_RELAX)
                if (relaxed) {
                    const Real *xc = (const Real *)((const unsigned char *)xb + (size_t)((t - 1) & 1) * xpar);
                    if constexpr (is_pms(CK)) relaxed_product<Real, CK, RG>(a, i, xc, z, img, prow_r[e], pcnt_r[e]);
                    else relaxed_product<Real, CK, RG>(a, i, xc, z);
                }
            const Real hh = WIDE_ELL ? (Real)0 : hv ? hv[i] : (Real)0;  // fixed-width rows: in y
            SW word = 0;
            // The replicas' updates.  A replica stopped by the convergence test keeps its angle,
            // moments and vertex; until one has stopped (always, without the test) the loop runs
            // without that per-replica test, whose branches would keep the compiler from
            // interleaving the replicas' updates.
            auto replicas = [&](auto check) __attribute__((always_inline)) {
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                const int k = e * RG + r;
                Real x = 0, c;
                Real sg;
                if constexpr (WIDE_ELL) {
                    // the fixed-width-row form: the vertex sign is the lane's own byte of the read
                    // parity; cos(theta) drives the update, sin(theta) only the loss (LOSS)
                    sg = (Real)(int)*(LdsI8 *)(size_t)tw_pos(RPc, e);
                    c = wrapped_cos(th[k]);
                    if constexpr (LOSS) {
                        Real cunused;
                        dsincos(th[k], &x, &cunused);
                    }
                } else {
                    if (KEEP) {
                        x = xs[k];
                        c = cs[k];
                    } else {
                        dsincos(th[k], &x, &c);
                    }
                    // s = sgn(sin theta) as +-1 (the vertex bit k of cur); products with it are exact
                    sg = x < 0 ? (Real)-1 : (Real)1;
                }
                const Real yh = WIDE_ELL ? y[r] : y[r] + hh;  // fixed-width rows: the field is in y
                Ep[r] = dfma(sg, yh, Ep[r]);
                Real tt = dfma(-mu, sg, yh);  // y - mu s + h
                if constexpr (WIDE_ELL) {
                    if constexpr (LOSS) Lp[r] = dfma(x, tt, Lp[r]);
                } else if constexpr (CAN_RELAX) {
                    if (relaxed) {
                        const Real zm = dfma(-mu, x, z[r]);  // z - mu x
                        tt = zm + hh;                                 // L term: z - mu x + h
                        Lp[r] = dfma(x, tt, Lp[r]);
                        tt = tt + zm;                                 // gradient term: 2 z - 2 mu x + h
                    } else {
                        Lp[r] = dfma(x, tt, Lp[r]);
                    }
                } else {
                    Lp[r] = dfma(x, tt, Lp[r]);
                }
                Real xn = x;  // a stopped replica keeps its angle, moments and vertex
                bool xneg = WIDE_ELL ? sg < 0 : x < 0;
                if (!decltype(check)::value || !((done >> r) & 1u)) {
                    Real tn;
                    if constexpr (WIDE_ELL) {
                        tn = angle_step_scaled(th[k], mo[k], ve[k], c * tt, adam, b1, b2, sa1, lr, sa2, eps);
                        // the wrap changes no angle below 3 in magnitude: it runs when some lane of
                        // the wavefront has a larger one (a uniform branch), else the sign is tn's
                        xneg = tn < (Real)0;
                        if (__builtin_amdgcn_ballot_w64((tn < (Real)0 ? -tn : tn) >= (Real)3)) {
                            tn = wrap_angle(tn);
                            xneg = wrapped_sin_neg(tn);
                        }
                    } else {
                        tn = angle_step(th[k], mo[k], ve[k], c * tt, adam, b1, omb1, b2, omb2, lib1, lr, ib2, eps);
                    }
                    th[k] = tn;
                    if constexpr (WIDE_ELL) {
                        // (its sign is set above)
                    } else if (KEEP) {
                        Real cn;
                        dsincos(tn, &xn, &cn);
                        xs[k] = xn;
                        cs[k] = cn;
                        xneg = xn < 0;
                    } else if (CAN_RELAX && relaxed) {
                        xn = dsin(tn);
                        xneg = xn < 0;
                    } else {
                        xneg = wrapped_sin_neg(tn);  // only the next vertex is needed
                    }
                }
                if constexpr (WIDE_ELL) {
                    word = xneg ? (SW)1 : (SW)0;
                } else if (xneg) {
                    nxt |= 1u << k;
                    word |= (SW)(1u << SWd::shift(r));
                }
                if (CAN_RELAX && relaxed) putx(t & 1, e * B + tid, r, xn);
            }
            };
            if constexpr (RG == 1) {
                // one replica: nothing to interleave (and without the loss no convergence test)
                if constexpr (WIDE_ELL && !LOSS) replicas(Flag<false>{});
                else replicas(Flag<true>{});
            } else {
                if (done) replicas(Flag<true>{});
                else replicas(Flag<false>{});
            }
            put(RPc >= 0 ? 1 - RPc : (t & 1), e, word);
            // keep the scheduler from interleaving elements: bounds live ranges
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            Ep[r] = wave_sum(Ep[r]);
            if (trace_l || conv) Lp[r] = wave_sum(Lp[r]);
        }
        if (lane == 0) {
            Real *epo = ep + ((t & 1) * NW + wave) * RG;
            Real *lpo = lp + ((t & 1) * NW + wave) * RG;
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                epo[r] = Ep[r];
                lpo[r] = Lp[r];
            }
        }
        __syncthreads();
        const uint32_t f = TWIN ? 0u : flg[(t - 1) & 1];
        if (f) {
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                if ((f >> r) & 1u) {
                    uint32_t mask = 0;
#pragma unroll
                    for (int e = 0; e < EPT; ++e) mask |= 1u << (e * RG + r);
                    best = (best & ~mask) | (prv & mask);
                }
            }
        }
        prv = cur;
        cur = nxt;
        if (TWIN || wave == 0) {
            bool imp = false;
            if (lane < RG) {
                Real Es = 0, Ls = 0;
                if constexpr (TWIN) {
                    // a fixed number of wavefronts (one replica): the partials load together, then
                    // add in wavefront order as below
                    constexpr int NWc = LB / 64;
                    Real pe[NWc], pl[NWc];
#pragma unroll
                    for (int w = 0; w < NWc; ++w) {
                        pe[w] = ep[(t & 1) * NWc + w];
                        if constexpr (LOSS) pl[w] = lp[(t & 1) * NWc + w];
                    }
#pragma unroll
                    for (int w = 0; w < NWc; ++w) {
                        Es += pe[w];
                        if constexpr (LOSS) Ls += pl[w];
                    }
                } else {
                    for (int w = 0; w < NW; ++w) {
                        Es += ep[((t & 1) * NW + w) * RG + lane];
                        Ls += lp[((t & 1) * NW + w) * RG + lane];
                    }
                }
                const double E = (double)Es, L = (double)Ls;
                imp = E < ebest && !((done >> lane) & 1u);  // a stopped replica is no longer scored
                if (imp) {
                    ebest = E;
                    bstep = a.t0 + t;
                }
                if (wave == 0) {
                    if (a.etrace) a.etrace[(size_t)(t - 1) * a.R + r0 + lane] = E;
                    if (trace_l) a.ltrace[(size_t)(t - 1) * a.R + r0 + lane] = L;
                }
            }
            const uint64_t bal = __ballot(imp);
            if constexpr (TWIN) twimp = bal != 0;  // one replica per workgroup
            else if (lane == 0) flg[t & 1] = (uint32_t)bal;
        }
        if (conv) {
            // every wavefront replays the test on the same loss (same order of summation as
            // above), so all of them agree on which replicas stop after this step
            bool now = false;
            if (lane < RG && !((done >> lane) & 1u)) {
                Real Ls = 0;
                for (int w = 0; w < NW; ++w) Ls += lp[((t & 1) * NW + w) * RG + lane];
                const int W = a.conv_window, tg = a.t0 + t;  // the test runs on the global step
                if (tg == 1) cring[kConvWindowMax * RG + lane] = Ls;
                cring[((tg - 1) % W) * RG + lane] = Ls;
                if (tg >= W) {
                    double mx = -INFINITY, mn = INFINITY;
                    for (int q = 0; q < W; ++q) {
                        const double v = (double)cring[q * RG + lane];
                        mx = fmax(mx, v);
                        mn = fmin(mn, v);
                    }
                    const double L1 = (double)cring[kConvWindowMax * RG + lane];
                    now = mx - mn <= a.conv_tol * fabs((double)Ls - L1);
                }
                if (now) conv_t = tg;
            }
            done |= (uint32_t)__ballot(now);
            if (done == (1u << RG) - 1u) {  // every replica of this workgroup has stopped
                tlast = t;
                return true;
            }
        }
        return false;
    };
    if constexpr (TWIN) {
        // two steps per iteration, each with its parity as a compile-time constant
        for (int t = 1; t <= a.steps; t += 2) {
            if (step(IntC<0>{}, t)) break;
            if (t + 1 > a.steps) break;
            if (step(IntC<1>{}, t + 1)) break;
        }
    } else {
        for (int t = 1; t <= a.steps; ++t)
            if (step(IntC<-1>{}, t)) break;
    }
    __syncthreads();
    if (a.conv_step && wave == 0 && lane < RG) a.conv_step[r0 + lane] = conv_t;
    if (conv && a.conv_state && wave == 0 && lane < RG) {
        Real *cs = (Real *)a.conv_state + (size_t)(r0 + lane) * (kConvWindowMax + 1);
        for (int q = 0; q <= kConvWindowMax; ++q) cs[q] = cring[q * RG + lane];
    }
    if constexpr (TWIN) {
        // the vertex scored in the last step, s^(tlast-1), is in parity (tlast - 1) & 1
        if (tlast > 0 && twimp) tw_keep((tlast - 1) & 1);
    } else if (tlast > 0) {
        const uint32_t f = flg[tlast & 1];
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            if ((f >> r) & 1u) {
                uint32_t mask = 0;
#pragma unroll
                for (int e = 0; e < EPT; ++e) mask |= 1u << (e * RG + r);
                best = (best & ~mask) | (prv & mask);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        if (e * B + tid >= n) continue;
        const int i = local_index<EPT>(spin_of(e));
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const int k = e * RG + r;
            const size_t idx = (size_t)(r0 + r) * n + i;
            gth[idx] = th[k];
            if (gm) gm[idx] = CK == CK_PME ? mo[k] * (Real)(1.0 - a.b1) : mo[k];
            if (gv) gv[idx] = CK == CK_PME ? ve[k] * (Real)(1.0 - a.b2) : ve[k];
            a.s_best[idx] = ((best >> k) & 1u) ? (int8_t)-1 : (int8_t)1;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (wave == 0 && lane < RG) {
        a.e_best[r0 + lane] = ebest;
        a.best_step[r0 + lane] = bstep;
    }
}


// Split-step form of the staged-image engine for four replicas per workgroup and one spin
// per thread (FP32, vertex loss, no field, exact integer sums; no traces or convergence test).
// With one spin per thread the 4 n (spin, replica) updates of a workgroup would run on
// ceil(n / 64) wavefronts, 4 of them on one SIMD for n = 800, which then sets the step time.
// Here a step is
//   A: thread q < n computes y of position q for the four replicas from the staged image
//      (as the engine does) and puts them in LDS;
//   B: all 1024 threads update (position, replica) items j = k 1024 + thread, each thread
//      always the same replica (j mod 4), so the updates spread evenly over 16 wavefronts.
// The vertex bytes are written where the engine writes its words and the energy sums are exact
// integers in any order.  No loss is computed here, so an item's update is that of the
// fixed-width-row form without the loss: cos(theta) alone (wrapped_cos), the sign of the vertex
// kept as +-1, scaled moments, and the wrap only where some lane of the wavefront needs it; its
// rounding differs from the engine's (which evaluates sin and cos together), and both are
// compared with the oracle.
constexpr int kSplitBlock = 1024, kSplitItems = 4;

size_t split_lds_bytes(int pms_rb, int pimg_groups, int bimg) {
    size_t off = ((size_t)4 * pms_rb + 15) & ~(size_t)15;
    off += (size_t)2 * (kSplitBlock / 64) * 4 * sizeof(float) + 8;
    off = (off + 15) & ~(size_t)15;
    off += (size_t)8 * pimg_groups;
    off = (off + 15) & ~(size_t)15;
    return off + (size_t)bimg * 4 * sizeof(float);
}

template <bool ADAM>  // the optimizer as a compile-time choice: no per-item branch
__global__ __launch_bounds__(kSplitBlock) void k_ds_split(const DSArgs a, int bimg) {
    constexpr int RG = 4, NW = kSplitBlock / 64, KI = kSplitItems;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = a.n, r0 = blockIdx.x * RG;
    const int rr = tid & 3;  // this thread's replica in every item
    size_t off = ((size_t)4 * a.pms_rb + 15) & ~(size_t)15;
    float *ep = (float *)(smem + off);  // [2][NW][RG]
    uint32_t *flg = (uint32_t *)(ep + 2 * NW * RG);
    off = (off + (size_t)2 * NW * RG * sizeof(float) + 8 + 15) & ~(size_t)15;
    uint2 *img = (uint2 *)(smem + off);
    off = (off + (size_t)8 * a.pimg_groups + 15) & ~(size_t)15;
    float *yb = (float *)(smem + off);  // [bimg][RG]
    auto vbuf = [&](int par) -> uint32_t * { return (uint32_t *)(smem + (size_t)par * 2 * a.pms_rb); };
    auto put_byte = [&](int par, int q, int r, bool neg) {
        unsigned char *w = (unsigned char *)vbuf(par);
        w[4 * q + r] = neg ? 1 : 0;               // field r of the word (one bit per replica)
        w[a.pms_rb + 4 * q + r] = neg ? 0 : 1;    // and of its complement
    };
    {
        const uint2 *src = (const uint2 *)a.pimg;
        for (int q = tid; q < a.pimg_groups; q += kSplitBlock) img[q] = src[q];
    }
    int prow = 0;
    uint32_t pcnt = 0;
    if (tid < n) {
        prow = a.prow[tid];
        pcnt = a.pcnt[tid];
    }
    if (tid == 0) {
        vbuf(0)[bimg] = 0;
        vbuf(1)[bimg] = 0;
    }
    float *gth = (float *)a.theta, *gm = (float *)a.m, *gv = (float *)a.v;
    constexpr bool adam = ADAM;
    // per item: the angle, the moments scaled as in the fixed-width-row form (mo = m / (1 - b1),
    // ve = v / (1 - b2)) and the current vertex sign s as +-1
    float th[KI], mo[KI], ve[KI], sgn[KI];
    int spin[KI];
    uint32_t cur = 0, prv = 0, best = 0;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int j = k * kSplitBlock + tid;
        th[k] = mo[k] = ve[k] = 0.f;
        sgn[k] = 1.f;
        spin[k] = 0;
        if (j >= 4 * n) continue;
        const int q = j >> 2, i = a.pperm[q];
        spin[k] = i;
        const size_t idx = (size_t)(r0 + rr) * n + i;
        float t;
        if (a.init_mode == 0) {
            t = gth[idx];
            if (t > 3.15f || t < -3.15f) {  // angles the engines write are within pi_f
                const float qw = drint(t * Consts<float>::inv_twopi);
                t = t - qw * Consts<float>::twopi_hi;
                t = t - qw * Consts<float>::twopi_lo;
            }
            if (gm) mo[k] = gm[idx] / (float)(1.0 - a.b1);
            if (gv) ve[k] = gv[idx] / (float)(1.0 - a.b2);
            if (a.s_best[idx] < 0) best |= 1u << k;
        } else {
            const float u = a.init_mode == 1 ? ((const float *)a.uniform)[idx] : draw_uniform<float>(a.seed, r0 + rr, i);
            t = dasin(u);
        }
        th[k] = t;
        float x, c;
        dsincos(t, &x, &c);
        sgn[k] = x < 0 ? -1.f : 1.f;
        if (x < 0) cur |= 1u << k;
        put_byte(0, q, rr, x < 0);
    }
    if (tid < 2) flg[tid] = 0;
    double ebest = INFINITY;
    int bstep = 0;
    if (wave == 0 && lane < RG && a.init_mode == 0) {
        ebest = a.e_best[r0 + lane];
        bstep = a.best_step[r0 + lane];
    }
    __syncthreads();

    const float lr = (float)a.lr, mu = (float)a.mu, b1 = (float)a.b1, b2 = (float)a.b2, eps = (float)a.eps;
    const float omb1 = (float)(1.0 - a.b1), omb2 = (float)(1.0 - a.b2);
    const float *bct = (const float *)a.bias;
    for (int t = 1; t <= a.steps; ++t) {
        const uint32_t *sc = vbuf((t - 1) & 1);
        const float ib1 = adam ? bct[2 * (t - 1)] : 1.f, ib2 = adam ? bct[2 * (t - 1) + 1] : 1.f;
        const float sa1 = lr * ib1 * omb1, sa2 = ib2 * omb2;  // the scaled-moment form's factors
        // A: the coupling product of position tid for the four replicas
        if (tid < n) {
            float y[RG];
            coupling<float, CK_PMS, RG>(a, 0, sc, y, img, prow, pcnt);
            *(float4 *)(yb + 4 * tid) = make_float4(y[0], y[1], y[2], y[3]);
        }
        __syncthreads();
        // B: the items' updates
        float Ep = -0.f;
        uint32_t nxt = 0;
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int j = k * kSplitBlock + tid;
            if (j >= 4 * n) continue;
            const int q = j >> 2;
            // cos(theta) alone drives the update (no loss is computed here); the sign of the
            // vertex is kept as +-1
            const float c = wrapped_cos(th[k]);
            const float sg = sgn[k];
            const float yh = yb[j];  // no field
            Ep = dfma(sg, yh, Ep);
            const float tt = dfma(-mu, sg, yh);
            float tn = angle_step_scaled(th[k], mo[k], ve[k], c * tt, adam, b1, b2, sa1, lr, sa2, eps);
            // the wrap changes no angle below 3 in magnitude: it runs when some lane of the
            // wavefront has a larger one (a uniform branch), else the sign is tn's
            bool neg = tn < 0.f;
            if (__builtin_amdgcn_ballot_w64(__builtin_fabsf(tn) >= 3.f)) {
                tn = wrap_angle(tn);
                neg = wrapped_sin_neg(tn);
            }
            th[k] = tn;
            sgn[k] = neg ? -1.f : 1.f;
            if (neg) nxt |= 1u << k;
            put_byte(t & 1, q, rr, neg);
        }
        // per-replica sums (exact integers: any order): the four lanes of a replica in each row of
        // 16 lanes by two DPP rotations, then across the four rows by two lane exchanges
        Ep += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, Ep), 0x124, 0xF, 0xF, false));
        Ep += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, Ep), 0x128, 0xF, 0xF, false));
        Ep += __shfl_xor(Ep, 16);
        Ep += __shfl_xor(Ep, 32);
        if (lane < RG) ep[((t & 1) * NW + wave) * RG + lane] = Ep;
        __syncthreads();
        if ((flg[(t - 1) & 1] >> rr) & 1u) best = prv;
        prv = cur;
        cur = nxt;
        if (wave == 0) {
            bool imp = false;
            if (lane < RG) {
                float Es = 0;
                for (int w = 0; w < NW; ++w) Es += ep[((t & 1) * NW + w) * RG + lane];
                const double E = (double)Es;
                imp = E < ebest;
                if (imp) {
                    ebest = E;
                    bstep = a.t0 + t;
                }
            }
            const uint64_t bal = __ballot(imp);
            if (lane == 0) flg[t & 1] = (uint32_t)bal;
        }
    }
    __syncthreads();
    if (a.steps > 0 && ((flg[a.steps & 1] >> rr) & 1u)) best = prv;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int j = k * kSplitBlock + tid;
        if (j >= 4 * n) continue;
        const size_t idx = (size_t)(r0 + rr) * n + spin[k];
        gth[idx] = th[k];
        if (gm) gm[idx] = mo[k] * (float)(1.0 - a.b1);
        if (gv) gv[idx] = ve[k] * (float)(1.0 - a.b2);
        a.s_best[idx] = ((best >> k) & 1u) ? (int8_t)-1 : (int8_t)1;
    }
    if (wave == 0 && lane < RG) {
        a.e_best[r0 + lane] = ebest;
        a.best_step[r0 + lane] = bstep;
    }
}

template <typename Real, int CK, int RG, int EPT, int OPT = -1, bool LOSS = true, bool PLAIN = false, int LBX = 0>
__global__ __launch_bounds__(LBX > 0 ? LBX : launch_bound(EPT)) void k_ds(const DSArgs a) {
    ds_body<Real, CK, RG, EPT, OPT, LOSS, PLAIN, LBX>(a, blockIdx.x * RG);
}

// Batched form for serving: workgroup b runs replica group map[b].y of problem
// map[b].x; every problem's steps and state are independent of the others'.
template <typename Real, int CK, int RG, int EPT>
__global__ __launch_bounds__(launch_bound(EPT)) void k_ds_batch(const DSArgs *descs, const int2 *map) {
    const int2 m = map[blockIdx.x];
    ds_body<Real, CK, RG, EPT>(descs[m.x], m.y * RG);
}

// Same step for problems too large to keep the state in registers: angles and
// moments are streamed from global memory every step (each workgroup touches
// only its own replicas, so there is still no inter-workgroup dependence), and
// the vertex is triple-buffered in LDS so that s_{t-1} is still readable when
// the best-vertex decision of step t-1 arrives.
template <typename Real, int CK, int RG>
__global__ __launch_bounds__(1024) void k_ds_stream(const DSArgs a) {
    using SWd = SpinWord<RG>;
    using SW = typename SWd::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, B = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, NW = B >> 6;
    SW *sbuf = (SW *)smem;  // [3][n]
    const size_t off = ((size_t)3 * n * sizeof(SW) + 15) & ~(size_t)15;
    Real *ep = (Real *)(smem + off);
    Real *lp = ep + 2 * NW * RG;
    uint32_t *flg = (uint32_t *)(lp + 2 * NW * RG);
    const int r0 = blockIdx.x * RG;
    const Real *hv = (const Real *)a.h;
    Real *gth = (Real *)a.theta;
    Real *gm = (Real *)a.m;
    Real *gv = (Real *)a.v;
    const bool adam = a.opt == ISING_OPT_ADAM;

    // buffer k % 3 holds s_{t0+k}; the initial vertex is s_{t0+1}... use local step t: buf[t % 3] = s_t
    for (int i = tid; i < n; i += B) {
        SW word = 0;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const size_t idx = (size_t)(r0 + r) * n + i;
            Real t;
            if (a.init_mode == 0) {
                t = gth[idx];
                if (t > (Real)3.5 || t < (Real)-3.5) {  // angles this engine wrote are within pi
                    const Real qw = drint(t * Consts<Real>::inv_twopi);
                    t = t - qw * Consts<Real>::twopi_hi;
                    t = t - qw * Consts<Real>::twopi_lo;
                    gth[idx] = t;  // the steps read the angle back from memory
                }
            } else {
                const Real u = a.init_mode == 1 ? ((const Real *)a.uniform)[idx]
                                                : draw_uniform<Real>(a.seed, r0 + r, i);
                t = dasin(u);
                gth[idx] = t;
                if (gm) gm[idx] = 0;
                if (gv) gv[idx] = 0;
                a.s_best[idx] = 1;
            }
            if (dsin_neg(t)) word |= (SW)(1u << SWd::shift(r));
        }
        sbuf[1 * n + i] = word;
    }
    if (tid < 2) flg[tid] = 0;
    double ebest = INFINITY;
    int bstep = 0;
    if (wave == 0 && lane < RG && a.init_mode == 0) {
        ebest = a.e_best[r0 + lane];
        bstep = a.best_step[r0 + lane];
    }
    __syncthreads();
    const Real lr = (Real)a.lr, mu = (Real)a.mu, b1 = (Real)a.b1, b2 = (Real)a.b2, eps = (Real)a.eps;
    const Real omb1 = (Real)(1.0 - a.b1), omb2 = (Real)(1.0 - a.b2);
    const Real *bct = (const Real *)a.bias;
    const bool trace_l = a.ltrace != nullptr;

    auto apply_best = [&](uint32_t f, const SW *sold) {
        for (int i = tid; i < n; i += B) {
            const uint32_t wd = (uint32_t)sold[i];
#pragma unroll
            for (int r = 0; r < RG; ++r)
                if ((f >> r) & 1u)
                    a.s_best[(size_t)(r0 + r) * n + i] = ((wd >> SWd::shift(r)) & 1u) ? (int8_t)-1 : (int8_t)1;
        }
    };

    for (int t = 1; t <= a.steps; ++t) {
        const SW *sc = sbuf + (t % 3) * n;
        SW *sn = sbuf + ((t + 1) % 3) * n;
        const Real ib1 = adam ? bct[2 * (t - 1)] : (Real)1, ib2 = adam ? bct[2 * (t - 1) + 1] : (Real)1;
        Real Ep[RG], Lp[RG];
#pragma unroll
        for (int r = 0; r < RG; ++r) Ep[r] = Lp[r] = 0;
        for (int i = tid; i < n; i += B) {
            Real y[RG];
            coupling<Real, CK, RG>(a, i, sc, y);
            const Real hh = hv ? hv[i] : (Real)0;
            const uint32_t wcur = (uint32_t)sc[i];
            SW word = 0;
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                const size_t idx = (size_t)(r0 + r) * n + i;
                const bool neg = (wcur >> SWd::shift(r)) & 1u;
                const Real yh = y[r] + hh;
                Ep[r] += neg ? -yh : yh;
                const Real tt = neg ? yh + mu : yh - mu;
                const Real th = gth[idx];
                Real x, c;
                dsincos(th, &x, &c);
                Lp[r] += x * tt;
                const Real g = c * tt;
                Real upd;
                if (adam) {
                    const Real mo = b1 * gm[idx] + omb1 * g;
                    const Real ve = b2 * gv[idx] + omb2 * (g * g);
                    gm[idx] = mo;
                    gv[idx] = ve;
                    upd = lr * (mo * ib1) * drcp(dsqrt(ve * ib2) + eps);
                } else {
                    upd = lr * g;
                }
                Real tn = th - upd;
                const Real q = drint(tn * Consts<Real>::inv_twopi);
                tn = tn - q * Consts<Real>::twopi_hi;
                tn = tn - q * Consts<Real>::twopi_lo;
                gth[idx] = tn;
                if (wrapped_sin_neg(tn)) word |= (SW)(1u << SWd::shift(r));
            }
            sn[i] = word;
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            Ep[r] = wave_sum(Ep[r]);
            if (trace_l) Lp[r] = wave_sum(Lp[r]);
        }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                ep[((t & 1) * NW + wave) * RG + r] = Ep[r];
                lp[((t & 1) * NW + wave) * RG + r] = Lp[r];
            }
        }
        __syncthreads();
        const uint32_t f = flg[(t - 1) & 1];
        if (f) apply_best(f, sbuf + ((t - 1) % 3) * n);
        if (wave == 0) {
            bool imp = false;
            if (lane < RG) {
                Real Es = 0, Ls = 0;
                for (int w = 0; w < NW; ++w) {
                    Es += ep[((t & 1) * NW + w) * RG + lane];
                    Ls += lp[((t & 1) * NW + w) * RG + lane];
                }
                const double E = (double)Es, L = (double)Ls;
                imp = E < ebest;
                if (imp) {
                    ebest = E;
                    bstep = a.t0 + t;
                }
                if (a.etrace) a.etrace[(size_t)(t - 1) * a.R + r0 + lane] = E;
                if (a.ltrace) a.ltrace[(size_t)(t - 1) * a.R + r0 + lane] = L;
            }
            const uint64_t bal = __ballot(imp);
            if (lane == 0) flg[t & 1] = (uint32_t)bal;
        }
    }
    __syncthreads();
    if (a.steps > 0) {
        const uint32_t f = flg[a.steps & 1];
        if (f) apply_best(f, sbuf + (a.steps % 3) * n);
    }
    if (wave == 0 && lane < RG) {
        a.e_best[r0 + lane] = ebest;
        a.best_step[r0 + lane] = bstep;
    }
}

// 1/(1 - b1^t) and 1/(1 - b2^t) for t = t0+1 .. t0+steps, in FP64, rounded to Real
template <typename Real>
__global__ void k_bias_table(double b1, double b2, int t0, int steps, Real *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= steps) return;
    const double t = (double)(t0 + q + 1);
    out[2 * q] = (Real)(1.0 / -expm1(t * log(b1)));
    out[2 * q + 1] = (Real)(1.0 / -expm1(t * log(b2)));
}

template <typename Real>
__global__ void k_format(DevProblem p, int packed, uint32_t *pm, Real *val_out, Real *h_out) {
    const int64_t total = p.format == ISING_DENSE ? (int64_t)p.n * p.n : p.nnz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const void *src = p.format == ISING_DENSE ? p.J : p.val;
        double v;
        if (p.vtype == ISING_I32) v = ((const int32_t *)src)[q];
        else if (p.vtype == ISING_F32) v = ((const float *)src)[q];
        else v = ((const double *)src)[q];
        if (packed) pm[q] = (uint32_t)p.col[q] | (v < 0 ? 0x80000000u : 0u);
        else val_out[q] = (Real)v;
    }
    if (h_out && p.h) {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p.n;
             i += (int64_t)gridDim.x * blockDim.x) {
            double v;
            if (p.vtype == ISING_I32) v = ((const int32_t *)p.h)[i];
            else if (p.vtype == ISING_F32) v = ((const float *)p.h)[i];
            else v = ((const double *)p.h)[i];
            h_out[i] = (Real)v;
        }
    }
}

// Fixed-width neighbour rows for the wide engine, one 16-byte record per position q = e * block + t
// (spin q): its (at most four) entries 2 col + (J < 0), the byte of the neighbour's term sgn(J) s in
// the vertex buffer; unused entries 2 ept block, the zero pair.  hrow[q]: the spin's field in FP32
// (0 without one, and for q >= n).
__global__ void k_ell_format(DevProblem p, const uint32_t *pm, const float *hf, int ept, int block, uint32_t *ell,
                             float *hrow) {
    const int total = ept * block;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int e = q / block, t = q % block;
        const int rs = q < p.n ? p.row_ptr[q] : 0, deg = q < p.n ? p.row_ptr[q + 1] - rs : 0;
        uint32_t *o = ell + ((size_t)e * block + t) * kEllWidth;
#pragma unroll
        for (int j = 0; j < kEllWidth; ++j)
            o[j] = j < deg ? 2u * (pm[rs + j] & 0x7fffffffu) + (pm[rs + j] >> 31) : 2u * (uint32_t)total;
        hrow[(size_t)e * block + t] = hf && q < p.n ? hf[q] : 0.f;
    }
}

// Sign-split LDS image of +-w couplings: per row, J > 0 neighbours then J < 0
// neighbours (ascending columns), each run padded to a multiple of 4 with the
// byte offset of the zero vertex word; entries are byte offsets col * wbytes.
// ---- staged +-w image (CK_PMS) -------------------------------------------

template <typename V>
__device__ inline double csr_value(const DevProblem &p, int q) {
    return (double)((const V *)p.val)[q];
}
__device__ inline double csr_value_any(const DevProblem &p, int q) {
    if (p.vtype == ISING_I32) return csr_value<int32_t>(p, q);
    if (p.vtype == ISING_F32) return csr_value<float>(p, q);
    return csr_value<double>(p, q);
}

// entries a coupling takes in the staged image: |v| / w for couplings that are integer
// multiples of the unit w (one for the common magnitude of +-w problems)
__device__ inline int pms_multiplicity(double v, double wunit) {
    return v == 0.0 ? 0 : (int)rint(fabs(v) / wunit);
}

// entries of each row (its degree counted with multiplicity)
__global__ void k_pms_degree(DevProblem p, double wunit, int32_t *deg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    int d = 0;
    for (int q = p.row_ptr[i]; q < p.row_ptr[i + 1]; ++q) d += pms_multiplicity(csr_value_any(p, q), wunit);
    deg[i] = d;
}

// position of each row in the thread layout: decreasing degree, ties by index
__global__ __launch_bounds__(256) void k_pms_rank(int n, const int32_t *deg, int32_t *pos, int32_t *perm) {
    __shared__ int tile[1024];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int di = i < n ? deg[i] : 0;
    int rank = 0;
    for (int base = 0; base < n; base += 1024) {
        __syncthreads();
        for (int j = threadIdx.x; j < 1024; j += blockDim.x) tile[j] = base + j < n ? deg[base + j] : -1;
        __syncthreads();
        const int m = min(1024, n - base);
        for (int j = 0; j < m; ++j) {
            const int dj = tile[j];
            rank += (dj > di) || (dj == di && base + j < i);
        }
    }
    if (i < n) {
        pos[i] = rank;
        perm[rank] = i;
    }
}

// One workgroup.  Unit u = (e, w) is the wavefront w of element e: positions
// e * B + 64 w + lane.  Its group count is the largest ceil(deg / 4) of its rows;
// units are laid out one after another, group-major inside a unit.
__global__ __launch_bounds__(256) void k_pms_units(int n, int B, int units, const int32_t *deg,
                                                   const int32_t *perm, int32_t *prow, uint32_t *pcnt,
                                                   int32_t *total) {
    __shared__ int gsz[256];
    const int u = threadIdx.x;
    const int nw = B / 64;
    int g = 0;
    if (u < units) {
        const int q0 = (u / nw) * B + (u % nw) * 64;
        for (int l = 0; l < 64; ++l)
            if (q0 + l < n) g = max(g, (deg[perm[q0 + l]] + 3) >> 2);
    }
    gsz[u] = g;
    __syncthreads();
    if (u == 0) {
        int acc = 0;
        for (int v = 0; v < units; ++v) {
            const int c = gsz[v];
            gsz[v] = acc;
            acc += 64 * c;
        }
        *total = acc;
    }
    __syncthreads();
    if (u < units) {
        const int q0 = (u / nw) * B + (u % nw) * 64;
        for (int l = 0; l < 64; ++l) {
            const int q = q0 + l;
            const int d = q < n ? deg[perm[q]] : 0;
            prow[q] = gsz[u] + l;
            pcnt[q] = (uint32_t)d | ((uint32_t)g << 16);
        }
    }
}

// Neighbour order of the staged image.  The LDS serves a wavefront's reads in two
// halves of 32 lanes over 32 banks, so each half-wavefront of rows is scheduled on
// its own (workgroup 2u + h: rows 32h .. 32h + 31 of unit u).  Slot by slot and
// row by row, a row takes the remaining entry that costs least given the words
// the earlier rows of its half already read at that slot: nothing if it is the
// same word (a broadcast), else the number of distinct words already in its bank;
// ties go to the lowest remaining index.  Row j at slot m depends only on row j
// at slot m - 1 and rows < j at slot m, so the pairs (j, m) are taken along
// anti-diagonals j + m = d, all rows of a diagonal at once, with the bank state
// kept per slot.  An entry is the byte offset of the neighbour's word, in the
// complement region when J < 0; slots past a row's degree read the zero word.
// Rows with more than kPmsSchedMax entries keep CSR order.
constexpr int kPmsSchedMax = 128;

__global__ __launch_bounds__(256) void k_pms_fill(DevProblem p, double wunit, int slots, int block, int wbytes,
                                                  int rb, const int32_t *pos, const int32_t *perm,
                                                  const int32_t *prow, const uint32_t *pcnt, uint16_t *img) {
    __shared__ uint16_t ent[32][kPmsSchedMax];    // remaining entries of each row
    __shared__ int rem[32];                        // their count (-1: row kept in CSR order)
    __shared__ uint32_t bank_words[kPmsSchedMax][32];  // per slot and bank: first two distinct words
    __shared__ uint8_t bank_count[kPmsSchedMax][32];   // and the number of distinct words
    __shared__ uint16_t res[kPmsSchedMax][32];     // entry chosen for each slot and row
    const int nw = block / 64, u = blockIdx.x >> 1, h = blockIdx.x & 1;
    const int q0 = (u / nw) * block + (u % nw) * 64 + 32 * h;  // first position of this half
    const int t = threadIdx.x, j = t >> 3, s = t & 7;          // 8 lanes per row
    const int G = (int)(pcnt[q0] >> 16);
    const int S = min(4 * G, kPmsSchedMax);
    const uint16_t zero = (uint16_t)(wbytes * slots);
    const int q = q0 + j;
    uint16_t *out = img + (size_t)prow[q] * 4;  // slot m at out[(m / 4) * 256 + m % 4]
    // stage each row's nonzero entries in CSR order; rows too long are written here directly
    {
        int d = 0;
        const int deg = q < p.n ? (int)(pcnt[q] & 0xffffu) : 0;
        if (q < p.n) {
            const int i = perm[q];
            const int rs = p.row_ptr[i], re = p.row_ptr[i + 1];
            for (int c = rs; c < re; c += 8) {
                const int e = c + s;
                int mult = 0;
                uint16_t o = 0;
                if (e < re) {
                    const double v = csr_value_any(p, e);
                    mult = pms_multiplicity(v, wunit);
                    o = v > 0 ? (uint16_t)(wbytes * pos[p.col[e]]) : (uint16_t)(rb + wbytes * pos[p.col[e]]);
                }
                // inclusive prefix of the multiplicities over the row's 8 lanes
                int incl = mult;
                for (int off = 1; off < 8; off <<= 1) {
                    const int y = __shfl_up(incl, off, 8);
                    if (s >= off) incl += y;
                }
                const int k0 = d + incl - mult;
                for (int u = 0; u < mult; ++u) {
                    const int k = k0 + u;
                    if (deg <= kPmsSchedMax) ent[j][k] = o;
                    else out[(size_t)(k >> 2) * 256 + (k & 3)] = o;
                }
                d += __shfl(incl, 7, 8);
            }
            if (deg > kPmsSchedMax)
                for (int m = d + s; m < 4 * G; m += 8) out[(size_t)(m >> 2) * 256 + (m & 3)] = zero;
        }
        if (s == 0) rem[j] = deg > kPmsSchedMax ? -1 : d;
    }
    for (int x = t; x < S * 32; x += 256) bank_count[x >> 5][x & 31] = 0;
    __syncthreads();
    for (int dg = 0; dg < 32 + S - 1; ++dg) {
        const int m = dg - j;
        const int r = rem[j];
        const bool act = m >= 0 && m < S && r >= 0;
        uint32_t key = 0xffffffffu;
        if (act) {
            for (int e = s; e < r; e += 8) {
                const uint16_t o = ent[j][e];
                const int b = (o >> 2) & 31;
                const uint32_t c = bank_count[m][b], w = bank_words[m][b];
                const bool same = (c >= 1 && o == (w & 0xffffu)) || (c >= 2 && o == (w >> 16));
                key = min(key, ((same ? 0u : c) << 16) | (uint32_t)e);
            }
        }
        // minimum over the row's 8 lanes (an aligned half-row)
        key = min(key, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)key, 0xB1, 0xF, 0xF, false));
        key = min(key, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)key, 0x4E, 0xF, 0xF, false));
        key = min(key, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)key, 0x141, 0xF, 0xF, false));
        if (act && s == 0) {
            uint16_t o = zero;
            if (r > 0) {
                const int e = (int)(key & 0xffffu);
                o = ent[j][e];
                ent[j][e] = ent[j][r - 1];
                rem[j] = r - 1;
                const int b = (o >> 2) & 31;
                const uint32_t c = bank_count[m][b], w = bank_words[m][b];
                const bool same = (c >= 1 && o == (w & 0xffffu)) || (c >= 2 && o == (w >> 16));
                if (!same) {
                    if (c == 0) bank_words[m][b] = o;
                    else if (c == 1) bank_words[m][b] = w | ((uint32_t)o << 16);
                    bank_count[m][b] = (uint8_t)min(c + 1, 255u);
                }
            }
            res[m][j] = o;
        }
        __syncthreads();
    }
    // scheduled rows: slots past kPmsSchedMax (only when a long row set the unit's length) are zero
    if (rem[j] >= 0)
        for (int m = s; m < 4 * G; m += 8) out[(size_t)(m >> 2) * 256 + (m & 3)] = m < S ? res[m][j] : zero;
}

__global__ __launch_bounds__(1024) void k_select(const double *e, int R, int32_t *best) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    double bv = INFINITY;
    int bi = -1;
    for (int r = threadIdx.x; r < R; r += 1024) {
        const double x = e[r];
        if (bi < 0 || x < bv) {
            bv = x;
            bi = r;
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if (threadIdx.x < d) {
            const double ov = sv[threadIdx.x + d];
            const int oi = si[threadIdx.x + d];
            const double mv = sv[threadIdx.x];
            const int mi = si[threadIdx.x];
            const bool take = oi >= 0 && (mi < 0 || ov < mv || (ov == mv && oi < mi));
            if (take) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *best = si[0] < 0 ? 0 : si[0];
}

__global__ void k_gather_row(const int8_t *block, int n, const int32_t *best, int8_t *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = block[(size_t)(*best) * n + i];
}

using KFn = void (*)(const DSArgs);

template <typename Real, int CK, int RG>
KFn pick_ept(int ept) {
    switch (ept) {
        case 0:
            if constexpr (!is_pms(CK)) return k_ds_stream<Real, CK, RG>;
            return nullptr;
        case 1: return k_ds<Real, CK, RG, 1>;
        case 2: return k_ds<Real, CK, RG, 2>;
        case 4:
            if constexpr (RG <= 2) return k_ds<Real, CK, RG, 4>;
            return nullptr;
        // one replica per workgroup, up to 32 spins per thread (FP32, sparse couplings; the staged
        // image up to 8, where its per-spin row data still fits the registers)
        case 8:
            if constexpr (sizeof(Real) == 4 && RG == 1 && CK != CK_DENSE) return k_ds<Real, CK, RG, 8>;
            return nullptr;
        case 16:
            if constexpr (sizeof(Real) == 4 && RG == 1 && (CK == CK_PM || CK == CK_CSRV)) return k_ds<Real, CK, RG, 16>;
            return nullptr;
        case 28:
            if constexpr (sizeof(Real) == 4 && RG == 1 && (CK == CK_PM || CK == CK_CSRV)) return k_ds<Real, CK, RG, 28>;
            return nullptr;
        case 32:
            if constexpr (sizeof(Real) == 4 && RG == 1 && (CK == CK_PM || CK == CK_CSRV)) return k_ds<Real, CK, RG, 32>;
            return nullptr;
        default: return nullptr;
    }
}

template <typename Real, int CK>
KFn pick_rg(int rg, int ept) {
    if constexpr (sizeof(Real) == 8) {
        return rg == 1 ? pick_ept<Real, CK, 1>(ept) : nullptr;
    } else {
        switch (rg) {
            case 1: return pick_ept<Real, CK, 1>(ept);
            case 2: return pick_ept<Real, CK, 2>(ept);
            case 4: return pick_ept<Real, CK, 4>(ept);
            default: return nullptr;
        }
    }
}

// workgroup sizes of the fixed-width-row form: launch_bound(ept), or the small-problem blocks
bool pme_block_ok(int ept, int block) {
    return block == launch_bound(ept) || (block == kPmeSmallBlock && (ept == 4 || ept == 8));
}

template <typename Real>
KFn pick(int ck, int rg, int ept, bool adam, bool loss, bool plain, int block) {
    switch (ck) {
        case CK_PM: return pick_rg<Real, CK_PM>(rg, ept);
        case CK_PMS: return ept > 0 ? pick_rg<Real, CK_PMS>(rg, ept) : nullptr;
        case CK_PMSR: return ept > 0 ? pick_rg<Real, CK_PMSR>(rg, ept) : nullptr;
        case CK_PME:
            if constexpr (sizeof(Real) == 4) {
                if (rg != 1) return nullptr;
                // the optimizer compiled in (these kernels run the longest per launch), whether the
                // loss is needed (a trace or the convergence test), and unit couplings without a field
#define ISING_PME(E, LBX)                                                                                 \
    if (ept == E && block == (LBX > 0 ? LBX : launch_bound(E))) {                                          \
        if (loss) return adam ? k_ds<Real, CK_PME, 1, E, 1, true, false, LBX> : k_ds<Real, CK_PME, 1, E, 0, true, false, LBX>; \
        if (plain) return adam ? k_ds<Real, CK_PME, 1, E, 1, false, true, LBX> : k_ds<Real, CK_PME, 1, E, 0, false, true, LBX>; \
        return adam ? k_ds<Real, CK_PME, 1, E, 1, false, false, LBX> : k_ds<Real, CK_PME, 1, E, 0, false, false, LBX>; \
    }
                ISING_PME(8, 0)
                ISING_PME(16, 0)
                ISING_PME(28, 0)
                ISING_PME(32, 0)
                ISING_PME(4, kPmeSmallBlock)
                ISING_PME(8, kPmeSmallBlock)
#undef ISING_PME
            }
            return nullptr;
        case CK_CSRV: return pick_rg<Real, CK_CSRV>(rg, ept);
        case CK_DENSE: return pick_rg<Real, CK_DENSE>(rg, ept);
        default: return nullptr;
    }
}

}  // namespace

int ds_block_limit(int ept) { return ept > 0 ? launch_bound(ept) : 1024; }

int pme_small_ept(int n) { return n <= 4 * kPmeSmallBlock ? 4 : n <= 8 * kPmeSmallBlock ? 8 : 0; }

int32_t ds_max_n(bool fp64) {
    // streaming engine, one replica per workgroup: three byte-per-spin LDS buffers
    (void)fp64;
    return 48 * 1024;
}

hipError_t launch_ell_format(const DevProblem &p, const uint32_t *pm, const float *hf, int ept, int block,
                             uint32_t *ell, float *hrow, hipStream_t s) {
    if (p.format != ISING_CSR || ept <= 0 || !pme_block_ok(ept, block) || (int64_t)ept * block < p.n)
        return hipErrorInvalidValue;
    const int total = ept * block;
    hipLaunchKernelGGL(k_ell_format, dim3((total + 255) / 256), dim3(256), 0, s, p, pm, hf, ept, block, ell, hrow);
    return hipGetLastError();
}

hipError_t launch_ds_format(const DevProblem &p, bool fp64, bool packed, uint32_t *pm, void *val_out,
                            void *h_out, hipStream_t s) {
    const int64_t total = p.format == ISING_DENSE ? (int64_t)p.n * p.n : p.nnz;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((std::max<int64_t>(total, p.n) + 255) / 256, 8192));
    if (fp64)
        hipLaunchKernelGGL(k_format<double>, dim3(blocks), dim3(256), 0, s, p, packed ? 1 : 0, pm,
                           (double *)val_out, (double *)h_out);
    else
        hipLaunchKernelGGL(k_format<float>, dim3(blocks), dim3(256), 0, s, p, packed ? 1 : 0, pm,
                           (float *)val_out, (float *)h_out);
    return hipGetLastError();
}

hipError_t launch_ds(const DSArgs &a, const DSLaunch &l, hipStream_t s, std::string *kernel) {
    const int ck = l.coupling == CK_PMS && l.relaxed ? CK_PMSR
                 : l.coupling == CK_PM && a.ell != nullptr && !l.relaxed ? CK_PME
                                                                          : l.coupling;
    const bool adam = a.opt == ISING_OPT_ADAM;
    const bool need_loss = a.ltrace != nullptr || a.conv_tol > 0;
    const bool plain = ck == CK_PME && !need_loss && a.h == nullptr && a.w == 1.0;
    KFn fn = l.fp64 ? pick<double>(ck, l.rg, l.ept, adam, need_loss, plain, l.block)
                    : pick<float>(ck, l.rg, l.ept, adam, need_loss, plain, l.block);
    if (!fn) return hipErrorInvalidValue;
    if (l.block % 64 || l.block < 64 || l.block > ds_block_limit(l.ept) || (l.ept > 0 && (int64_t)l.ept * l.block < a.n) ||
        a.R % l.rg)
        return hipErrorInvalidValue;
    if (ck == CK_PME && (!pme_block_ok(l.ept, l.block) || !a.ellh))  // its positions assume B = its block
        return hipErrorInvalidValue;
    if (l.coupling == CK_PMS && a.pms_rb != pms_region_bytes(l)) return hipErrorInvalidValue;
    if ((a.loss == ISING_LOSS_RELAXED) != l.relaxed || (l.relaxed && l.ept <= 0))
        return hipErrorInvalidValue;
    if (ck == CK_PMS && !l.fp64 && l.rg == 4 && l.ept == 1 && a.exact_sums && !a.etrace && !a.ltrace &&
        a.conv_tol <= 0 && !a.conv_step && l.block <= kSplitBlock) {
        // the split-step form (same results, updates spread over all 16 wavefronts)
        const size_t lds = split_lds_bytes(a.pms_rb, a.pimg_groups, l.block);
        if (lds <= 160 * 1024) {
            const auto fn = a.opt == ISING_OPT_ADAM ? k_ds_split<true> : k_ds_split<false>;
            if (lds > 64 * 1024) {
                hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(fn, dim3(a.R / 4), dim3(kSplitBlock), lds, s, a, l.block);
            if (kernel) *kernel = a.opt == ISING_OPT_ADAM ? "k_ds_split<adam>" : "k_ds_split<gd>";
            return hipGetLastError();
        }
    }
    const size_t lds = ds_lds_bytes(l, a.n, a.pimg_groups, ck == CK_PME);
    const size_t lds_static = ck == CK_PME ? (size_t)2 * twin_stride(l.ept, l.block) : 0;
    if (lds + lds_static > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(a.R / l.rg), dim3(l.block), lds, s, a);
    if (kernel) {
        static const char *const cks[] = {"PM", "CSRV", "DENSE", "PMS", "PMSR", "PME"};
        const char *ckn = ck >= 0 && ck < (int)(sizeof(cks) / sizeof(cks[0])) ? cks[ck] : "?";
        *kernel = std::string(l.ept > 0 ? "k_ds<" : "k_ds_stream<") + (l.fp64 ? "double" : "float") + ", " + ckn +
                  ", rg=" + std::to_string(l.rg) + ", ept=" + std::to_string(l.ept) +
                  (ck == CK_PME && l.block != launch_bound(l.ept) ? ", block=" + std::to_string(l.block) : "") +
                  (ck == CK_PME ? (need_loss ? ", loss" : plain ? ", no loss, unit" : ", no loss") : "") + ">";
    }
    return hipGetLastError();
}

using KBFn = void (*)(const DSArgs *, const int2 *);

template <int CK>
KBFn pick_batch(int rg, int ept) {
    if (rg == 1) {
        if (ept == 1) return k_ds_batch<float, CK, 1, 1>;
        if (ept == 2) return k_ds_batch<float, CK, 1, 2>;
        if (ept == 4) return k_ds_batch<float, CK, 1, 4>;
    } else if (rg == 2) {
        if (ept == 1) return k_ds_batch<float, CK, 2, 1>;
        if (ept == 2) return k_ds_batch<float, CK, 2, 2>;
        if (ept == 4) return k_ds_batch<float, CK, 2, 4>;
    } else if (rg == 4) {
        if (ept == 1) return k_ds_batch<float, CK, 4, 1>;
        if (ept == 2) return k_ds_batch<float, CK, 4, 2>;
    }
    return nullptr;
}

hipError_t launch_ds_batch(const DSArgs *descs, const int2 *map, int nwg, const DSLaunch &l, size_t lds,
                           hipStream_t s) {
    if (l.fp64 || l.ept <= 0 || nwg <= 0) return hipErrorInvalidValue;
    KBFn fn = l.coupling == CK_PMS ? pick_batch<CK_PMS>(l.rg, l.ept)
            : l.coupling == CK_PM  ? pick_batch<CK_PM>(l.rg, l.ept)
            : l.coupling == CK_CSRV ? pick_batch<CK_CSRV>(l.rg, l.ept)
                                    : pick_batch<CK_DENSE>(l.rg, l.ept);
    if (!fn) return hipErrorInvalidValue;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(nwg), dim3(l.block), lds, s, descs, map);
    return hipGetLastError();
}

hipError_t launch_bias_table(double b1, double b2, int t0, int steps, bool fp64, void *out, hipStream_t s) {
    if (steps <= 0) return hipSuccess;
    if (fp64) hipLaunchKernelGGL(k_bias_table<double>, dim3((steps + 255) / 256), dim3(256), 0, s, b1, b2, t0, steps, (double *)out);
    else hipLaunchKernelGGL(k_bias_table<float>, dim3((steps + 255) / 256), dim3(256), 0, s, b1, b2, t0, steps, (float *)out);
    return hipGetLastError();
}

int pms_region_bytes(const DSLaunch &l) {
    const int wbytes = l.rg == 1 ? 1 : 4;
    return ((l.ept * l.block + 1) * wbytes + 255) / 256 * 256;
}

hipError_t launch_pms_format(const DevProblem &p, const DSLaunch &l, double wunit, PmsWork &w,
                             int32_t *total_groups, hipStream_t s) {
    const int slots = l.ept * l.block, units = slots / 64;
    if (l.ept <= 0 || slots < p.n || units > 256) return hipErrorInvalidValue;
    const dim3 g((p.n + 255) / 256);
    if (!w.img) {
        hipLaunchKernelGGL(k_pms_degree, g, dim3(256), 0, s, p, wunit, w.deg);
        hipLaunchKernelGGL(k_pms_rank, g, dim3(256), 0, s, p.n, w.deg, w.pos, w.perm);
        hipLaunchKernelGGL(k_pms_units, dim3(1), dim3(256), 0, s, p.n, l.block, units, w.deg, w.perm, w.prow,
                           w.pcnt, w.total);
        hipError_t e = hipMemcpyAsync(total_groups, w.total, 4, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    const int wbytes = l.rg == 1 ? 1 : 4;
    hipLaunchKernelGGL(k_pms_fill, dim3(2 * units), dim3(256), 0, s, p, wunit, slots, l.block, wbytes,
                       pms_region_bytes(l), w.pos, w.perm, w.prow, w.pcnt, w.img);
    return hipGetLastError();
}

size_t ds_lds_bytes(const DSLaunch &l, int n, int pimg_groups, bool twin) {
    const size_t sw = l.rg == 1 ? 1 : 4;
    const size_t real = l.fp64 ? 8 : 4;
    const int nw = l.block / 64;
    size_t sbytes;
    if (l.coupling == CK_PMS) sbytes = (size_t)4 * pms_region_bytes(l);
    else if (twin) sbytes = 0;  // static: twin_lds, 2 twin_stride(ept, block) bytes
    else sbytes = l.ept > 0 ? (size_t)2 * (l.ept * l.block + 1) * sw : (size_t)3 * n * sw;
    size_t lds = ((sbytes + 15) & ~(size_t)15) + 2 * 2 * nw * l.rg * real + 8;
    if (l.coupling == CK_PMS) lds = ((lds + 15) & ~(size_t)15) + (size_t)8 * pimg_groups;
    if (l.relaxed) {
        // sin(theta) double-buffered; CK_PMS: records at XS = rg * real / word bytes times the word
        // offsets, with a negated copy
        const size_t xs = (size_t)l.rg * real / sw;
        lds = ((lds + 15) & ~(size_t)15) + (l.coupling == CK_PMS ? (size_t)4 * xs * pms_region_bytes(l)
                                                                   : (size_t)2 * (l.ept * l.block + 1) * l.rg * real);
    }
    if (l.conv) lds = ((lds + 15) & ~(size_t)15) + (size_t)nw * (kConvWindowMax + 1) * l.rg * real;
    return lds;
}

hipError_t launch_select(const double *e_best, int32_t R, int32_t *best, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, e_best, R, best);
    return hipGetLastError();
}

hipError_t launch_gather_row(const int8_t *block, int32_t n, const int32_t *best, int8_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_row, dim3((n + 255) / 256), dim3(256), 0, s, block, n, best, out);
    return hipGetLastError();
}

}  // namespace ising
