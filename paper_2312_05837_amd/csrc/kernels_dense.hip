// Domain selection for dense couplings on the matrix cores (paper Sec. III-B).
//
// One launch per step: Y = J S~ (rows = spins, columns = replicas) on MFMA,
// then the step's elementwise update fused into the tile epilogue while the
// accumulators are still in registers:
//   E_r partial += s (y + h),  L_r partial += sin(theta) (y - mu s + h),
//   GD / ADAM update of theta, wrap, next vertex S~' = sgn(sin theta') written
//   as the next step's B operand.
// The per-row-tile energy partials of a step are combined in a fixed order, each
// replica's best energy kept and the vertex of an improvement copied by the next
// step's tiles (after their own epilogue; partials double-buffered by step parity,
// vertices in three buffers), and for the last step by a small second kernel.
//
// Forms of the coupling product (the iterates are FP32 in all of them):
//   DF_FP32   J and S~ in FP32, v_mfma_f32_32x32x2_f32
//   DF_BF16X2 J = J_hi + J_lo, both BF16 (J_hi = bf16(J), J_lo = bf16(J - J_hi)),
//             S~ = +-1 exact in BF16, two v_mfma_f32_32x32x16_bf16 per k-step
//             into the same FP32 accumulators
//   DF_BF16   J_hi only
//   DF_FP8    couplings of one integer magnitude w: J / w = -1, 0, +1 and the vertex
//             exact in FP8 (E4M3), v_mfma_f32_32x32x64_f8f6f4, y = w (J / w) S~ exact
//   DF_I8X3   J = 2^e Jq with Jq an integer of three balanced INT8 digits (Jq = 65536 a +
//   DF_I8X2   256 b + c; two digits for I8X2, one for I8X1, which FP32 requests on integer
//   DF_I8X1   couplings up to 127 run: exact there) and one power-of-two scale for the whole
//             matrix; the vertex +-1 in INT8; v_mfma_i32_32x32x32_i8 digit plane by digit
//             plane with the accumulators multiplied by 256 between planes (Horner), so
//             Jq S~ is exact in int32 and y = 2^e float(Jq S~) rounds once.  e is the
//             smallest exponent with max|J| <= 2^e qmax (qmax = 127 (256^D - 1) / 255)
//             and max_i sum_j |J_ij| + 2^e 257 n <= 2^e (2^31 - 1), which bounds every
//             partial sum of every plane (any order) below 2^31.
// Tile: 128 spins x 128 replicas per workgroup of four wavefronts (2 x 2, each
// 64 x 64 = 2 x 2 MFMA blocks of 32 x 32); the split form and the INT8 forms of two and
// three digits 128 x 256 on eight (2 x 4).
// K staged through LDS in chunks of 64 BF16 / 128 FP8 or INT8 values (32 FP32); the INT8
// forms run their digit planes one after another through the same K loop.
// Operand layouts: J padded row-major [Mp][Kp]; S~ replica-major [R][Kp]
// (each replica's spins contiguous), so both MFMA operands are K-contiguous.
// State theta, m, v, s_best: replica-major [R][n].
#include <vector>

#include "internal.hpp"

namespace ising {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// forms with one-byte operands (FP8, INT8) and the digit planes of J per product
__host__ __device__ constexpr bool int8_form(int f) { return f == DF_I8X3 || f == DF_I8X2 || f == DF_I8X1; }
__host__ __device__ constexpr bool byte_form(int f) { return f == DF_FP8 || int8_form(f); }
__host__ __device__ constexpr int jdigits(int f) { return f == DF_I8X3 ? 3 : f == DF_I8X2 ? 2 : 1; }
// largest |Jq| of D balanced INT8 digits: 127 (256^D - 1) / 255
__host__ __device__ constexpr double jq_max(int D) { return D == 3 ? 8355711.0 : D == 2 ? 32639.0 : 127.0; }

constexpr int BM = 128, BN = 128, KC = 32;
constexpr int KCB = 64;       // K chunk of the BF16 forms: one 128-byte line per row and chunk
constexpr int AST = KCB;      // LDS row stride (bf16 elements) of the BF16 chunks (16-byte units swizzled)
constexpr int FST = KC + 1;   // LDS row stride (floats) for the FP32 form
constexpr int TST = BM + 4;   // LDS row stride (floats) of the transposed accumulator tile
constexpr int GEMM_LDS_FP32 = (BM + BN) * FST * 4;
constexpr int EPI_LDS = 64 * TST * 4;
constexpr int cmax(int x, int y) { return x > y ? x : y; }

// Tile of one workgroup: BM spins by BN replicas on NT threads, wavefronts WM x WN of 64 x 64
// each.  The split form moves twice the operand bytes of J per product, so its tiles are twice
// as wide (256 replicas, 8 wavefronts, LDS double-buffered: one workgroup per CU): each staged
// chunk of J then serves twice the replicas, which cuts the L2-to-CU operand traffic per product
// by a third.
// (one plane of one-byte operands, FP8 or INT8, runs faster on the 128 x 128 tiles)
__host__ __device__ constexpr bool wide_form(int f) { return f == DF_BF16X2 || f == DF_I8X3 || f == DF_I8X2; }
template <int FORM>
struct TileShape {
    static constexpr bool WIDE = wide_form(FORM);
    static constexpr int BN = WIDE ? 256 : 128;
    static constexpr int NT = WIDE ? 512 : 256;
    static constexpr int WN = BN / 64, WM = BM / 64;
    static_assert(WM * WN * 64 == NT, "one 64 x 64 block per wavefront");
};
__host__ __device__ constexpr int tile_bn(int form) { return wide_form(form) ? 256 : 128; }
__host__ __device__ constexpr int tile_threads(int form) { return wide_form(form) ? 512 : 256; }

// sum of each 16-lane row of a wavefront (quads, then half rows, then rows), result in every lane
__device__ inline float row_sum16(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
    return v;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also orders
// global memory, which makes every wavefront wait for all of its outstanding
// global loads at each barrier and so drains the operand prefetch of the K loop.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline unsigned short bf16_bits(float x) {
    // round to nearest even
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ inline float bf16_to_f(unsigned short b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
// FP8 (E4M3) bytes of -1, 0, +1 as the conversion instruction writes them, so that they are
// read back by the matrix cores in the same format
__device__ inline unsigned char fp8_of(float x) {
    return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
}

// float sin/cos for |x| <= 4 (same construction as the persistent engine's)
__device__ inline void fsincos(float x, float *s, float *c) {
    const float k = rintf(x * 0.636619772367581343f);
    float r = __builtin_fmaf(-k, 1.57079637050628662f, x);
    r = __builtin_fmaf(-k, -4.37113882867379300e-08f, r);
    r = __builtin_fmaf(-k, -1.71512451000588190e-15f, r);
    const float r2 = r * r;
    float ps = __builtin_fmaf(r2, 2.75573192239858907e-06f, -1.98412698412698413e-04f);
    ps = __builtin_fmaf(r2, ps, 8.33333333333333333e-03f);
    ps = __builtin_fmaf(r2, ps, -1.66666666666666667e-01f);
    const float sn = __builtin_fmaf(r * r2, ps, r);
    float pc = __builtin_fmaf(r2, -2.75573192239858907e-07f, 2.48015873015873016e-05f);
    pc = __builtin_fmaf(r2, pc, -1.38888888888888889e-03f);
    pc = __builtin_fmaf(r2, pc, 4.16666666666666667e-02f);
    pc = __builtin_fmaf(r2, pc, -0.5f);
    const float cn = __builtin_fmaf(r2, pc, 1.0f);
    const int q = (int)k & 3;
    const float a = (q & 1) ? cn : sn;
    const float b = (q & 1) ? sn : cn;
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}

// The sign of the sine that fsincos(x) returns, from its range reduction alone: in the odd
// quadrants the sine is +-cos(r) (|r| <= pi/4, never zero), in the even ones +-sin(r), whose
// polynomial keeps the sign of r.  Gives the same answer as fsincos(x) followed by x < 0.
__device__ inline bool fsin_neg(float x) {
    const float k = rintf(x * 0.636619772367581343f);
    float r = __builtin_fmaf(-k, 1.57079637050628662f, x);
    r = __builtin_fmaf(-k, -4.37113882867379300e-08f, r);
    r = __builtin_fmaf(-k, -1.71512451000588190e-15f, r);
    const int q = (int)k & 3;
    return q == 3 || (q == 0 && r < 0.f) || (q == 2 && r > 0.f);
}

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---- operand preparation ----------------------------------------------------

template <typename V>
__global__ void k_dense_split(DevProblem p, int Mp, int Kp, int form, unsigned short *Jhi, unsigned short *Jlo,
                              float *Jf, float *hf, const int32_t *jexp) {
    const int e = int8_form(form) ? *jexp : 0;
    if (hf && p.h)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += gridDim.x * blockDim.x)
            hf[i] = (float)((const V *)p.h)[i];
    const int64_t total = (int64_t)Mp * Kp;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / Kp), j = (int)(q % Kp);
        const double v = (i < p.n && j < p.n) ? (double)((const V *)p.J)[(size_t)i * p.n + j] : 0.0;
        if (form == DF_FP32) {
            Jf[q] = (float)v;
        } else if (form == DF_FP8) {
            // J / w is -1, 0 or +1 (the caller checked one integer magnitude w)
            ((unsigned char *)Jhi)[q] = fp8_of(v == 0.0 ? 0.f : (v < 0.0 ? -1.f : 1.f));
        } else if (int8_form(form)) {
            // Jq = rint(J / 2^e) (the scaling is exact) as balanced base-256 digits, most
            // significant digit in plane 0; |Jq| <= qmax, so the top digit is within [-128, 127]
            // (|J| above qmax 2^127, where no exponent fits, saturates at qmax)
            const int D = jdigits(form);
            const double qm = jq_max(D);
            int64_t jq = (int64_t)fmin(fmax(rint(ldexp(v, -e)), -qm), qm);
            for (int d = D - 1; d >= 0; --d) {
                const int64_t c = ((jq + 128) & 255) - 128;
                ((signed char *)Jhi)[(size_t)d * total + q] = (signed char)c;
                jq = (jq - c) / 256;
            }
        } else {
            const float vf = (float)v;
            const unsigned short hi = bf16_bits(vf);
            Jhi[q] = hi;
            if (form == DF_BF16X2) Jlo[q] = bf16_bits((float)(v - (double)bf16_to_f(hi)));
        }
    }
}

// INT8 forms: the largest |J_ij| and the largest row sum of |J_ij| (FP64), as the bit patterns of
// non-negative doubles, which order like unsigned integers, into mx[0] and mx[1] (zeroed before).
template <typename V>
__global__ __launch_bounds__(256) void k_dense_absmax(DevProblem p, unsigned long long *mx) {
    __shared__ double ss[4], sm[4];
    for (int i = blockIdx.x; i < p.n; i += gridDim.x) {
        double sum = 0.0, big = 0.0;
        for (int j = threadIdx.x; j < p.n; j += 256) {
            const double a = fabs((double)((const V *)p.J)[(size_t)i * p.n + j]);
            sum += a;
            big = fmax(big, a);
        }
        for (int o = 32; o > 0; o >>= 1) {
            sum += __shfl_xor(sum, o);
            big = fmax(big, __shfl_xor(big, o));
        }
        if ((threadIdx.x & 63) == 0) {
            ss[threadIdx.x >> 6] = sum;
            sm[threadIdx.x >> 6] = big;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const double rs = (ss[0] + ss[1]) + (ss[2] + ss[3]);
            const double rm = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
            atomicMax(mx + 0, (unsigned long long)__double_as_longlong(rm));
            atomicMax(mx + 1, (unsigned long long)__double_as_longlong(rs));
        }
        __syncthreads();
    }
}

// The scale exponent e of the INT8 forms (one thread): the smallest e with max|J| <= 2^e qmax and
// max row sum + 2^e 257 n <= 2^e (2^31 - 1), within [-126, 127] so that 2^e is a normal float.
// Writes 2^e (float) at byte 16 and e at byte 20 of the scale buffer.
__global__ void k_dense_exponent(int n, int digits, unsigned long long *mx) {
    const double big = __longlong_as_double((long long)mx[0]), rsum = __longlong_as_double((long long)mx[1]);
    const double qmax = jq_max(digits), lim = 2147483647.0;
    auto fits = [&](int e) { return big <= ldexp(qmax, e) && rsum + ldexp(257.0 * n, e) <= ldexp(lim, e); };
    int e = -126;
    if (big > 0.0) {
        int k;
        frexp(big / qmax, &k);
        e = max(-126, k - 2);
        while (e < 127 && !fits(e)) ++e;
        while (e > -126 && fits(e - 1)) --e;
    }
    float *f = (float *)((char *)mx + 16);
    *f = ldexpf(1.f, e);
    *(int32_t *)((char *)mx + 20) = e;
}

// theta_0 = asin(U), m = v = 0, S~_1 = sgn(sin theta_0) (padding zero), e_best = +inf
__global__ void k_dense_init(int n, int R, int Kp, int form, int init_mode, uint64_t seed, const float *uniform,
                             float *theta, float *m, float *v, void *S, void *S_other, void *S_third,
                             double *e_best, int32_t *best_step, int8_t *s_best) {
    const int64_t total = (int64_t)R * Kp;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(q / Kp), i = (int)(q % Kp);
        float s = 0.f;
        if (i < n) {
            const size_t idx = (size_t)r * n + i;
            float th;
            if (init_mode == 0) {
                th = theta[idx];
            } else {
                float u;
                if (init_mode == 1) {
                    u = uniform[idx];
                } else {
                    const uint64_t z = splitmix64(seed, ((uint64_t)(uint32_t)r << 32) | (uint32_t)i);
                    u = 2.f * ((float)(uint32_t)(z >> 40) * 5.9604644775390625e-08f) - 1.f;
                }
                th = asinf(u);
                theta[idx] = th;
                if (m) m[idx] = 0.f;
                if (v) v[idx] = 0.f;
                s_best[idx] = 1;
            }
            float x, c;
            fsincos(th, &x, &c);
            s = x < 0.f ? -1.f : 1.f;
        }
        if (form == DF_FP32) {
            ((float *)S)[q] = s;
            ((float *)S_other)[q] = 0.f;  // the other buffers' padding must be zero too
            ((float *)S_third)[q] = 0.f;
        } else if (byte_form(form)) {
            ((unsigned char *)S)[q] = form == DF_FP8 ? fp8_of(s) : (unsigned char)(signed char)s;
            ((unsigned char *)S_other)[q] = 0;
            ((unsigned char *)S_third)[q] = 0;
        } else {
            ((unsigned short *)S)[q] = bf16_bits(s);
            ((unsigned short *)S_other)[q] = 0;
            ((unsigned short *)S_third)[q] = 0;
        }
    }
    if (init_mode != 0) {
        for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
            e_best[r] = INFINITY;
            best_step[r] = 0;
        }
    }
}

// ---- the step ---------------------------------------------------------------

// Per-problem descriptor, constant over a chunk of steps: the step index tloc
// (1-based within the chunk) is the only per-launch argument, so every problem
// of a group advances with the same two launches per step.
template <typename T>
using plain_ptr = T *;
// pointer into device global memory: accesses through it compile to global
// (not flat) loads and stores
template <typename T>
using global_ptr = __attribute__((address_space(1))) T *;

template <template <typename> class Ptr>
struct DenseDescT {
    int n, R, Mp, Kp, opt, mtiles;
    float lr, mu, b1, b2, eps, omb1, omb2;
    int t0;                  // global step before the chunk
    float jscale;            // y = jscale * (J S~) of the stored operand (w for the FP8 form, else 1)
    Ptr<const float> jpow;   // INT8 forms: y = 2^e float(Jq S~), 2^e in device memory
    Ptr<const float> bias;   // 1/(1-b1^t), 1/(1-b2^t) of the chunk's steps, at 2 (tloc - 1)
    Ptr<const unsigned short> Jhi, Jlo;
    Ptr<const float> Jf;
    Ptr<const float> h;
    // vertex buffers: step tloc reads S[(tloc - 1) % 3] and writes S[tloc % 3] (S0 holds the
    // chunk's first vertex), so the vertex scored in step tloc - 1 is intact through step tloc
    Ptr<char> S0, S1, S2;
    Ptr<float> theta, m, v;
    Ptr<float> Epart, Lpart;  // [2][mtiles][R]: step tloc writes part tloc & 1
    Ptr<double> e_best;
    Ptr<int32_t> best_step;
    Ptr<int8_t> s_best;
    Ptr<double> etrace, ltrace;  // rows of the chunk's steps (nullable)
};
// written by the host; the kernels read the same bytes with global pointers
using DenseDesc = DenseDescT<plain_ptr>;
using DenseDescG = DenseDescT<global_ptr>;
static_assert(sizeof(DenseDesc) == sizeof(DenseDescG), "descriptor layouts must agree");

// One K chunk (64) of the BF16 operands held in registers: rows tid / 8 + (NT / 8) p of the J
// tile (hi, and lo for the split form; BM rows) and of the vertex tile (BN rows), 8 bf16 at
// 16-byte unit tid % 8.  Eight lanes read one row's 128-byte line of the chunk: the loads use
// whole cache lines (half lines with a chunk of 32 limit the misses a CU's vector cache holds).
template <int FORM>
struct BfStage {
    static constexpr int RS = TileShape<FORM>::NT / 8;  // rows per pass
    static constexpr int NA = BM / RS, NB = TileShape<FORM>::BN / RS;
    u16x8 ah[NA], al[NA], b[NB];
};
// Element offset of 16-byte unit u (8 bf16, u = 0..7) of row r in an LDS chunk.  The unit
// index is XORed with (r ^ (r >> 3)) & 7, so that the MFMA fragment reads (one row per
// lane, one unit) touch distinct banks.
__device__ __forceinline__ int swz(int r, int u) { return r * AST + ((u ^ r ^ (r >> 3)) & 7) * 8; }

// J rows start at plane offset joff (2-byte units; INT8 digit planes), the vertex rows at 0.
template <int FORM>
__device__ __forceinline__ BfStage<FORM> bf_gload(const DenseDescG &a, const void *S_in, int row0, int col0, int k0,
                                                  int tid, size_t joff = 0) {
    using St = BfStage<FORM>;
    St s;
    const int rr = tid >> 3, c8 = (tid & 7) * 8;
    const size_t kpu = byte_form(FORM) ? a.Kp >> 1 : a.Kp;  // row length in 2-byte units
    const unsigned short *Sb = (const unsigned short *)S_in;
#pragma unroll
    for (int p = 0; p < St::NA; ++p) {
        const size_t ja = joff + (size_t)(row0 + rr + St::RS * p) * kpu + k0 + c8;
        s.ah[p] = *(const u16x8 *)(a.Jhi + ja);
        s.al[p] = FORM == DF_BF16X2 ? *(const u16x8 *)(a.Jlo + ja) : u16x8{};
    }
#pragma unroll
    for (int p = 0; p < St::NB; ++p)  // replica rows past R read row R - 1 (no branch around the
                                      // load); the stage store writes zeros for them
        s.b[p] = *(const u16x8 *)(Sb + (size_t)min(col0 + rr + St::RS * p, a.R - 1) * kpu + k0 + c8);
    return s;
}
// the J part goes to Ah (hi) and Al (lo), the vertex part to Bs
template <int FORM>
__device__ __forceinline__ void bf_stage_store(unsigned short *Ah, unsigned short *Al, unsigned short *Bs,
                                               const BfStage<FORM> &s, int tid, int col0, int R) {
    using St = BfStage<FORM>;
    const int rr = tid >> 3, u = tid & 7;
#pragma unroll
    for (int p = 0; p < St::NA; ++p) {
        const int o = swz(rr + St::RS * p, u);
        *(u16x8 *)(Ah + o) = s.ah[p];
        if (FORM == DF_BF16X2) *(u16x8 *)(Al + o) = s.al[p];
    }
#pragma unroll
    for (int p = 0; p < St::NB; ++p)
        *(u16x8 *)(Bs + swz(rr + St::RS * p, u)) = col0 + rr + St::RS * p < R ? s.b[p] : u16x8{};
}

// vertex buffer k (0..2); the buffer addresses are selected as values (a select of the fields
// themselves makes the compiler keep the whole descriptor in scratch memory)
__device__ __forceinline__ char *vbuf(const DenseDescG &a, int k) {
    const uintptr_t p0 = (uintptr_t)(char *)a.S0, p1 = (uintptr_t)(char *)a.S1, p2 = (uintptr_t)(char *)a.S2;
    return (char *)(k == 0 ? p0 : k == 1 ? p1 : p2);
}

// Step tloc's energy of replica r from the row-tile partials (ascending tile order) and its
// best-vertex update; one wavefront (lane = 0..63).
__device__ __forceinline__ void best_of(const DenseDescG &a, const int tloc, const int r, const int lane, const int form) {
    const size_t ppar = (size_t)(tloc & 1) * a.mtiles * a.R;
    const void *S_t = (const void *)vbuf(a, (tloc - 1) % 3);
    // row-tile partials loaded by the lanes together, summed in ascending tile order
    float E = 0.f, L = 0.f;
    for (int t0 = 0; t0 < a.mtiles; t0 += 64) {
        const int t = t0 + lane;
        const float ev = t < a.mtiles ? a.Epart[ppar + (size_t)t * a.R + r] : 0.f;
        const float lv = (a.ltrace && t < a.mtiles) ? a.Lpart[ppar + (size_t)t * a.R + r] : 0.f;
        const int m = min(64, a.mtiles - t0);
        for (int j = 0; j < m; ++j) {
            E += __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, ev), j));
            L += __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, lv), j));
        }
    }
    const bool imp = (double)E < a.e_best[r];
    if (imp) {
        const size_t src = (size_t)r * a.Kp, dst = (size_t)r * a.n;
        if ((a.n & 7) == 0) {
            // 8 spins per lane and iteration: 16 (BF16) or 32 (FP32) bytes in, 8 bytes out
            for (int i = 8 * lane; i < a.n; i += 512) {
                float sv[8];
                if (form == DF_FP32) {
                    const float4 p0 = *(const float4 *)((const float *)S_t + src + i);
                    const float4 p1 = *(const float4 *)((const float *)S_t + src + i + 4);
                    sv[0] = p0.x; sv[1] = p0.y; sv[2] = p0.z; sv[3] = p0.w;
                    sv[4] = p1.x; sv[5] = p1.y; sv[6] = p1.z; sv[7] = p1.w;
                } else if (byte_form(form)) {
                    // the sign bit of an FP8 or INT8 value is its top bit
                    const uint2 p8 = *(const uint2 *)((const unsigned char *)S_t + src + i);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        sv[u] = (p8.x >> (8 * u + 7)) & 1 ? -1.f : 1.f;
                        sv[u + 4] = (p8.y >> (8 * u + 7)) & 1 ? -1.f : 1.f;
                    }
                } else {
                    const u16x8 p8 = *(const u16x8 *)((const unsigned short *)S_t + src + i);
#pragma unroll
                    for (int u = 0; u < 8; ++u) sv[u] = bf16_to_f(p8[u]);
                }
                uint32_t lo = 0, hi = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    lo |= (uint32_t)(uint8_t)(sv[u] < 0.f ? -1 : 1) << (8 * u);
                    hi |= (uint32_t)(uint8_t)(sv[u + 4] < 0.f ? -1 : 1) << (8 * u);
                }
                *(uint2 *)(a.s_best + dst + i) = make_uint2(lo, hi);
            }
        } else {
            for (int i = lane; i < a.n; i += 64) {
                const float sv = form == DF_FP32  ? ((const float *)S_t)[src + i]
                                 : byte_form(form) ? (((const unsigned char *)S_t)[src + i] & 0x80 ? -1.f : 1.f)
                                                  : bf16_to_f(((const unsigned short *)S_t)[src + i]);
                a.s_best[dst + i] = sv < 0.f ? (int8_t)-1 : (int8_t)1;
            }
        }
    }
    if (lane == 0) {
        if (imp) {
            a.e_best[r] = (double)E;
            a.best_step[r] = a.t0 + tloc;
        }
        if (a.etrace) a.etrace[(size_t)(tloc - 1) * a.R + r] = (double)E;
        if (a.ltrace) a.ltrace[(size_t)(tloc - 1) * a.R + r] = (double)L;
    }
}

template <int FORM>
__device__ __forceinline__ void dense_step_body(const DenseDescG &a, const int tloc, const int mt, const int nt) {
    using TS = TileShape<FORM>;
    constexpr int TBN = TS::BN, NTH = TS::NT;
    // split form: two buffers of J hi, vertex and J lo rows
    __shared__ __align__(16) unsigned char lds[cmax(FORM == DF_FP32    ? 2 * GEMM_LDS_FP32
                                                    : FORM == DF_BF16X2 ? 2 * (2 * BM + TBN) * AST * 2
                                                                        : 2 * (BM + TBN) * AST * 2,
                                                    EPI_LDS)];
    __shared__ float red_e[1][TBN], red_l[1][TBN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / TS::WN, wn = wave % TS::WN;
    const void *S_in = (const void *)vbuf(a, (tloc - 1) % 3);
    void *S_out = (void *)vbuf(a, tloc % 3);
    const float ib1 = a.opt == ISING_OPT_ADAM ? a.bias[2 * (tloc - 1)] : 1.f;
    const float ib2 = a.opt == ISING_OPT_ADAM ? a.bias[2 * (tloc - 1) + 1] : 1.f;
    const int row0 = mt * BM, col0 = nt * TBN;
    f32x16 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x16{};

    // K loop: the next chunk's global loads are issued into registers before the
    // current chunk's MFMAs, and LDS is double-buffered, so one barrier per chunk.
    const int nchunks = a.Kp / KC;
    if constexpr (FORM == DF_FP32) {
        float4 pa[4], pb[4];
        auto gload = [&](int k0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = tid + 256 * u;
                const int r = q / (KC / 4), c4 = (q % (KC / 4)) * 4;
                pa[u] = *(const float4 *)(a.Jf + (size_t)(row0 + r) * a.Kp + k0 + c4);
                pb[u] = (col0 + r < a.R) ? *(const float4 *)((const float *)S_in + (size_t)(col0 + r) * a.Kp + k0 + c4)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        gload(0);
        for (int c = 0; c < nchunks; ++c) {
            float *As = (float *)lds + (c & 1) * (BM + BN) * FST;
            float *Bs = As + BM * FST;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = tid + 256 * u;
                const int r = q / (KC / 4), c4 = (q % (KC / 4)) * 4;
                As[r * FST + c4] = pa[u].x; As[r * FST + c4 + 1] = pa[u].y;
                As[r * FST + c4 + 2] = pa[u].z; As[r * FST + c4 + 3] = pa[u].w;
                Bs[r * FST + c4] = pb[u].x; Bs[r * FST + c4 + 1] = pb[u].y;
                Bs[r * FST + c4 + 2] = pb[u].z; Bs[r * FST + c4 + 3] = pb[u].w;
            }
            lds_barrier();
            if (c + 1 < nchunks) gload((c + 1) * KC);
#pragma unroll
            for (int ks = 0; ks < KC; ks += 2) {
                const int kk = ks + (lane >> 5);
                float av[2], bv[2];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) av[bi] = As[(wm * 64 + bi * 32 + (lane & 31)) * FST + kk];
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) bv[bj] = Bs[(wn * 64 + bj * 32 + (lane & 31)) * FST + kk];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
            }
        }
    } else {
        // NST chunks in flight in registers (stages refilled in turn, NST chunks ahead), one
        // LDS-only barrier per chunk with two LDS buffers.  The global loads are issued
        // unconditionally (the last chunk is re-read) so that the wait for the oldest stage is
        // a fixed count of outstanding loads.
        constexpr int NST = 2;  // register budget: two workgroups per CU (one for the split form's wide tile)
        constexpr int BUF = FORM == DF_BF16X2 ? (2 * BM + TBN) * AST : (BM + TBN) * AST;  // bf16 elements
        // chunks of 128 bytes per row: 64 BF16 or 128 FP8 / INT8 values of k; the INT8 forms run
        // nch chunks per digit plane, planes in turn (chunk g: plane g / nch)
        const int nch = (byte_form(FORM) ? a.Kp >> 1 : a.Kp) / KCB, ntot = jdigits(FORM) * nch, last = ntot - 1;
        const size_t plane = (size_t)a.Mp * (a.Kp >> 1);  // 2-byte units per INT8 digit plane
        auto gl = [&](int g) {
            const int p = jdigits(FORM) == 1 ? 0 : (g >= nch) + (jdigits(FORM) == 3 && g >= 2 * nch);
            return bf_gload<FORM>(a, S_in, row0, col0, (g - p * nch) * KCB, tid, p * plane);
        };
        BfStage<FORM> s0 = gl(0);
        BfStage<FORM> s1 = gl(min(1, last));
        BfStage<FORM> s2;
        if (NST == 3) s2 = gl(min(2, last));
        // Chunk c's products from LDS buffer c & 1.  The stage holding chunk c + 1 is written to
        // the other buffer among the products (that buffer was last read by chunk c - 1, before
        // the previous barrier; after the last chunk it is written with a re-read chunk that no
        // one reads), so the LDS stores overlap the matrix cores instead of standing between two
        // barriers.  BF16 forms: the fragments of k-step ks + 1 are read while the products of
        // k-step ks run, and the scheduler is asked to interleave the stores with the products.
        auto chunk = [&](const int c, BfStage<FORM> &next) {
            const unsigned short *Ah = (const unsigned short *)lds + (c & 1) * BUF;
            const unsigned short *Bs = Ah + BM * AST;
            const unsigned short *Al = Bs + TBN * AST;
            unsigned short *Nh = (unsigned short *)lds + ((c + 1) & 1) * BUF;
            auto store = [&]() { bf_stage_store<FORM>(Nh, Nh + (BM + TBN) * AST, Nh + BM * AST, next, tid, col0, a.R); };
            if constexpr (byte_form(FORM)) {
                // 32 bytes (k 64 ks + 32 (l / 32) .. + 31) per lane and operand; both operands put
                // the same k in the same lane slot, so the k order inside the instruction is
                // immaterial (INT8: the first and second 16 bytes feed two 32-k products)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int u = 4 * ks + 2 * (lane >> 5);
                    i32x8 af[2], bf[2];
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi) {
                        const int r = wm * 64 + bi * 32 + (lane & 31);
                        const i32x4 lo = __builtin_bit_cast(i32x4, *(const u16x8 *)(Ah + swz(r, u)));
                        const i32x4 hi = __builtin_bit_cast(i32x4, *(const u16x8 *)(Ah + swz(r, u + 1)));
                        af[bi] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                    }
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) {
                        const int r = wn * 64 + bj * 32 + (lane & 31);
                        const i32x4 lo = __builtin_bit_cast(i32x4, *(const u16x8 *)(Bs + swz(r, u)));
                        const i32x4 hi = __builtin_bit_cast(i32x4, *(const u16x8 *)(Bs + swz(r, u + 1)));
                        bf[bj] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                    }
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj) {
                            if constexpr (FORM == DF_FP8) {
                                acc[bi][bj] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                    af[bi], bf[bj], acc[bi][bj], 0, 0, 0, 0, 0, 0);
                            } else {
                                const i32x4 a0 = {af[bi][0], af[bi][1], af[bi][2], af[bi][3]};
                                const i32x4 a1 = {af[bi][4], af[bi][5], af[bi][6], af[bi][7]};
                                const i32x4 b0 = {bf[bj][0], bf[bj][1], bf[bj][2], bf[bj][3]};
                                const i32x4 b1 = {bf[bj][4], bf[bj][5], bf[bj][6], bf[bj][7]};
                                i32x16 c = __builtin_bit_cast(i32x16, acc[bi][bj]);
                                c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, c, 0, 0, 0);
                                c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, c, 0, 0, 0);
                                acc[bi][bj] = __builtin_bit_cast(f32x16, c);
                            }
                        }
                    if (ks == 0) store();
                }
            } else {
                struct Frag {
                    bf16x8 ah[2], al[2], bv[2];
                };
                auto read = [&](int ks) {
                    Frag f;
                    const int u = 2 * ks + (lane >> 5);
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi) {
                        const int o = swz(wm * 64 + bi * 32 + (lane & 31), u);
                        f.ah[bi] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(Ah + o));
                        if (FORM == DF_BF16X2) f.al[bi] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(Al + o));
                    }
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        f.bv[bj] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(Bs + swz(wn * 64 + bj * 32 + (lane & 31), u)));
                    return f;
                };
                auto mfma = [&](const Frag &f) {
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj) {
                            if (FORM == DF_BF16X2)
                                acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.al[bi], f.bv[bj], acc[bi][bj], 0, 0, 0);
                            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[bi], f.bv[bj], acc[bi][bj], 0, 0, 0);
                        }
                };
                static_assert(KCB / 16 == 4, "four k-steps per chunk");
                constexpr int NMF = FORM == DF_BF16X2 ? 8 : 4;  // products per k-step
                constexpr int NWR = BfStage<FORM>::NA * (FORM == DF_BF16X2 ? 2 : 1) + BfStage<FORM>::NB;  // stores
                Frag f0 = read(0);
                Frag f1 = read(1);
                store();
                mfma(f0);
                f0 = read(2);
                mfma(f1);
                f1 = read(3);
                mfma(f0);
                mfma(f1);
                // order: the stores spread over the first two k-steps' products, each k-step's
                // fragment reads ahead of its products
#pragma unroll
                for (int q = 0; q < 2 * NMF; ++q) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one product
                    if (q < NWR) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // one LDS store
                }
            }
        };
        bf_stage_store<FORM>((unsigned short *)lds, (unsigned short *)lds + (BM + TBN) * AST,
                             (unsigned short *)lds + BM * AST, s0, tid, col0, a.R);
        s0 = gl(min(NST, last));
        lds_barrier();
        // INT8 forms, first chunk of a digit plane after the first: the accumulators hold the
        // higher digits' sum, which the next digit's terms join at 256 times its weight
        auto horner = [&](int g) {
            if (int8_form(FORM) && (g == nch || g == 2 * nch))
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        acc[bi][bj] = __builtin_bit_cast(f32x16, __builtin_bit_cast(i32x16, acc[bi][bj]) << 8);
        };
        // iteration c stores the stage of chunk c + 1 and refills it with chunk c + 1 + NST
#define DENSE_BF_CHUNK(C, ST)                                                                          \
    {                                                                                                  \
        const int c_ = (C);                                                                            \
        horner(c_);                                                                                    \
        chunk(c_, ST);                                                                                 \
        __builtin_amdgcn_sched_barrier(0);                                                             \
        ST = gl(min(c_ + 1 + NST, last));                                                              \
        lds_barrier();                                                                                 \
    }
        int c = 0;
        if constexpr (NST == 3) {
            for (; c + 3 <= ntot; c += 3) {
                DENSE_BF_CHUNK(c, s1);
                DENSE_BF_CHUNK(c + 1, s2);
                DENSE_BF_CHUNK(c + 2, s0);
            }
            if (c < ntot) DENSE_BF_CHUNK(c, s1);
            if (c + 1 < ntot) DENSE_BF_CHUNK(c + 1, s2);
        } else {
            for (; c + 2 <= ntot; c += 2) {
                DENSE_BF_CHUNK(c, s1);
                DENSE_BF_CHUNK(c + 1, s0);
            }
            if (c < ntot) DENSE_BF_CHUNK(c, s1);
        }
#undef DENSE_BF_CHUNK
    }
    lds_barrier();  // the epilogue reuses LDS

    // ---- fused epilogue.  The accumulators (C block (bi, bj), lane l, element q hold
    // row 64 wm + 32 bi + 8 (q / 4) + 4 (l / 32) + q % 4, column 64 wn + 32 bj + l % 32) are
    // transposed through LDS, 64 replica columns (one wavefront column) at a time, so that each
    // thread then owns 4 consecutive spins of a replica: the state streams as float4
    // with 32 lanes covering 128 consecutive spins of one replica.
    const bool adam = a.opt == ISING_OPT_ADAM;
    // the vertex bytes of +1 and -1 (FP8 or INT8)
    const unsigned char f8p = FORM == DF_FP8 ? fp8_of(1.f) : 1, f8m = FORM == DF_FP8 ? fp8_of(-1.f) : 0xff;
    const float jp = int8_form(FORM) ? *a.jpow : 1.f;  // 2^e
    float *T = (float *)lds;  // [64 replicas][TST]
    const int g = tid & 31;   // spin group: rows 4g .. 4g+3 of the tile
    const int i0 = row0 + 4 * g;
    const bool vec = (a.n & 3) == 0 && i0 + 3 < a.n;
    float h4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) h4[u] = (a.h && i0 + u < a.n) ? a.h[i0 + u] : 0.f;
    // The state of all KR replicas a thread updates in one part is loaded together (before the
    // accumulators are transposed), so that its loads are in flight together: the epilogue is
    // bound by this traffic.  Thread tid takes replicas tid / 32 + RSTEP k.  With 512 threads (KR
    // = 4) the next part's state is loaded while the current part is updated, two buffers, so
    // that as many loads stay in flight as with two 256-thread workgroups per CU.
    constexpr int RSTEP = NTH / 32, KR = 64 / RSTEP;
    constexpr int NSB = KR <= 4 ? 2 : 1;  // state buffers
    float sth_[NSB][KR][4], smo_[NSB][KR][4], sve_[NSB][KR][4];
    auto load_half = [&](int half) {
        float(&sth)[KR][4] = sth_[half % NSB];
        float(&smo)[KR][4] = smo_[half % NSB];
        float(&sve)[KR][4] = sve_[half % NSB];
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int r = col0 + half * 64 + (tid >> 5) + RSTEP * k;
#pragma unroll
            for (int u = 0; u < 4; ++u) sth[k][u] = smo[k][u] = sve[k][u] = 0.f;
            if (r < a.R && i0 < a.n) {
                const size_t base = (size_t)r * a.n + i0;
                if (vec) {
                    const float4 t4 = *(const float4 *)(a.theta + base);
                    sth[k][0] = t4.x; sth[k][1] = t4.y; sth[k][2] = t4.z; sth[k][3] = t4.w;
                    if (adam) {
                        const float4 m4 = *(const float4 *)(a.m + base);
                        const float4 v4 = *(const float4 *)(a.v + base);
                        smo[k][0] = m4.x; smo[k][1] = m4.y; smo[k][2] = m4.z; smo[k][3] = m4.w;
                        sve[k][0] = v4.x; sve[k][1] = v4.y; sve[k][2] = v4.z; sve[k][3] = v4.w;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool ok = i0 + u < a.n;
                        sth[k][u] = ok ? a.theta[base + u] : 0.f;
                        smo[k][u] = (ok && adam) ? a.m[base + u] : 0.f;
                        sve[k][u] = (ok && adam) ? a.v[base + u] : 0.f;
                    }
                }
            }
        }
    };
    if (NSB == 2) load_half(0);
#pragma unroll
    for (int half = 0; half < TS::WN; ++half) {
        if (NSB == 1) load_half(half);
        else if (half + 1 < TS::WN) load_half(half + 1);
        float(&sth)[KR][4] = sth_[half % NSB];
        float(&smo)[KR][4] = smo_[half % NSB];
        float(&sve)[KR][4] = sve_[half % NSB];
        if (wn == half) {
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int m = wm * 64 + bi * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                        const int nl = bj * 32 + (lane & 31);
                        T[nl * TST + m] = acc[bi][bj][q];
                    }
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int rl = (tid >> 5) + RSTEP * k;    // replica within this part
            const int r = col0 + half * 64 + rl;
            float th[4], mo[4], ve[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                th[u] = sth[k][u];
                mo[u] = smo[k][u];
                ve[u] = sve[k][u];
            }
            float Ep = 0.f, Lp = 0.f;
            if (r < a.R && i0 < a.n) {
                const float4 y4 = *(const float4 *)(T + rl * TST + 4 * g);
                float yv[4] = {y4.x, y4.y, y4.z, y4.w};
                if constexpr (FORM == DF_FP8)
#pragma unroll
                    for (int u = 0; u < 4; ++u) yv[u] *= a.jscale;  // exact: integers below 2^24
                if constexpr (int8_form(FORM))
#pragma unroll
                    for (int u = 0; u < 4; ++u) yv[u] = (float)__builtin_bit_cast(int, yv[u]) * jp;  // one rounding
                const size_t base = (size_t)r * a.n + i0;
                unsigned short sb[4];
                float sf[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    float x, c;
                    fsincos(th[u], &x, &c);
                    const bool neg = x < 0.f;
                    const float yh = yv[u] + h4[u];
                    const bool live = i0 + u < a.n;
                    Ep += live ? (neg ? -yh : yh) : 0.f;
                    const float tt = neg ? yh + a.mu : yh - a.mu;
                    Lp += live ? x * tt : 0.f;
                    const float gr = c * tt;
                    float upd;
                    if (adam) {
                        mo[u] = a.b1 * mo[u] + a.omb1 * gr;
                        ve[u] = a.b2 * ve[u] + a.omb2 * (gr * gr);
                        upd = a.lr * (mo[u] * ib1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(ve[u] * ib2) + a.eps);
                    } else {
                        upd = a.lr * gr;
                    }
                    float tn = th[u] - upd;
                    const float kq = rintf(tn * 0.159154943091895336f);
                    tn = tn - kq * 6.28318548202514648f;
                    tn = tn - kq * -1.7484555314695172e-07f;
                    th[u] = tn;
                    const bool nn = fsin_neg(tn);
                    sf[u] = live ? (nn ? -1.f : 1.f) : 0.f;
                    sb[u] = live ? (nn ? (unsigned short)0xBF80 : (unsigned short)0x3F80) : (unsigned short)0;  // bf16 of sf
                }
                if (vec) {
                    *(float4 *)(a.theta + base) = make_float4(th[0], th[1], th[2], th[3]);
                    if (adam) {
                        *(float4 *)(a.m + base) = make_float4(mo[0], mo[1], mo[2], mo[3]);
                        *(float4 *)(a.v + base) = make_float4(ve[0], ve[1], ve[2], ve[3]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (i0 + u < a.n) {
                            a.theta[base + u] = th[u];
                            if (adam) {
                                a.m[base + u] = mo[u];
                                a.v[base + u] = ve[u];
                            }
                        }
                }
                const size_t sbase = (size_t)r * a.Kp + i0;  // Kp % 64 == 0, i0 % 4 == 0: aligned
                if (FORM == DF_FP32) {
                    *(float4 *)((float *)S_out + sbase) = make_float4(sf[0], sf[1], sf[2], sf[3]);
                } else if (byte_form(FORM)) {
                    uint32_t w = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) w |= (uint32_t)(sf[u] == 0.f ? 0 : sf[u] < 0.f ? f8m : f8p) << (8 * u);
                    *(uint32_t *)((unsigned char *)S_out + sbase) = w;
                } else {
                    const uint2 w = make_uint2((uint32_t)sb[0] | ((uint32_t)sb[1] << 16),
                                               (uint32_t)sb[2] | ((uint32_t)sb[3] << 16));
                    *(uint2 *)((unsigned short *)S_out + sbase) = w;
                }
            }
            // sum over the 32 spin groups of this replica (lanes 0-31 and 32-63 hold two replicas):
            // quad, half-row and row sums by DPP, then the two rows of each half-wavefront
            Ep = row_sum16(Ep);
            Lp = row_sum16(Lp);
            const float e_lo = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Ep), 15)) +
                               __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Ep), 31));
            const float e_hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Ep), 47)) +
                               __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Ep), 63));
            const float l_lo = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Lp), 15)) +
                               __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Lp), 31));
            const float l_hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Lp), 47)) +
                               __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Lp), 63));
            if (lane == 0) {
                const int rw = half * 64 + (wave * 2) + RSTEP * k;  // replica of lanes 0-31 (tid >> 5 = 2 wave)
                red_e[0][rw] = e_lo;
                red_e[0][rw + 1] = e_hi;
                red_l[0][rw] = l_lo;
                red_l[0][rw + 1] = l_hi;
            }
        }
        lds_barrier();
    }
    const size_t ppar = (size_t)(tloc & 1) * a.mtiles * a.R;
    if (tid < TBN && col0 + tid < a.R) {
        a.Epart[ppar + (size_t)mt * a.R + col0 + tid] = red_e[0][tid];
        if (a.Lpart) a.Lpart[ppar + (size_t)mt * a.R + col0 + tid] = red_l[0][tid];
    }
    // The previous step's best-vertex bookkeeping for this tile's share of its replica columns
    // (its partials are complete: written by the previous launch), one wavefront per replica.
    if (tloc > 1) {
        const int share = (TBN + a.mtiles - 1) / a.mtiles;
        const int rb = col0 + mt * share, re = min(min(col0 + TBN, a.R), rb + share);
        for (int r = rb + wave; r < re; r += NTH / 64) best_of(a, tloc - 1, r, lane, FORM);
    }
}

// (two workgroups per CU for the 256-thread tiles: at most 256 registers per lane)
template <int FORM>
__global__ __launch_bounds__(TileShape<FORM>::NT, TileShape<FORM>::WIDE ? 1 : 2) void k_dense_step(
    const DenseDesc *__restrict__ descs,
                                                    const int4 *__restrict__ tiles, int tloc) {
    const int4 t = tiles[blockIdx.x];  // (problem, row tile, replica tile)
    const DenseDescG a = ((const DenseDescG *)descs)[t.x];
    dense_step_body<FORM>(a, tloc, t.y, t.z);
}

// one wavefront per replica: the last step of a chunk (earlier steps are kept by the next step's
// tiles)
__global__ __launch_bounds__(256) void k_dense_best(const DenseDesc *__restrict__ descs,
                                                    const int2 *__restrict__ quads, int tloc, int form) {
    const int2 qd = quads[blockIdx.x];  // (problem, group of four replicas)
    const DenseDescG a = ((const DenseDescG *)descs)[qd.x];
    const int r = qd.y * 4 + (threadIdx.x >> 6);
    if (r < a.R) best_of(a, tloc, r, threadIdx.x & 63, form);
}

}  // namespace

hipError_t launch_dense_prepare(const DevProblem &p, int form, int Mp, int Kp, void *Jhi, void *Jlo, void *Jf,
                                float *hf, void *jsc, hipStream_t s) {
    const int64_t total = (int64_t)Mp * Kp;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    const int32_t *jexp = nullptr;
    if (int8_form(form)) {
        if (!jsc) return hipErrorInvalidValue;
        // a fill kernel would do as well; this runs before any captured launch sequence
        hipError_t e = hipMemsetAsync(jsc, 0, 16, s);
        if (e != hipSuccess) return e;
        const int rb = std::min(p.n, 4096);
        unsigned long long *mx = (unsigned long long *)jsc;
        if (p.vtype == ISING_I32) hipLaunchKernelGGL(k_dense_absmax<int32_t>, dim3(rb), dim3(256), 0, s, p, mx);
        else if (p.vtype == ISING_F32) hipLaunchKernelGGL(k_dense_absmax<float>, dim3(rb), dim3(256), 0, s, p, mx);
        else hipLaunchKernelGGL(k_dense_absmax<double>, dim3(rb), dim3(256), 0, s, p, mx);
        hipLaunchKernelGGL(k_dense_exponent, dim3(1), dim3(1), 0, s, p.n, jdigits(form), mx);
        jexp = (const int32_t *)((const char *)jsc + 20);
    }
    if (p.vtype == ISING_I32)
        hipLaunchKernelGGL(k_dense_split<int32_t>, dim3(blocks), dim3(256), 0, s, p, Mp, Kp, form,
                           (unsigned short *)Jhi, (unsigned short *)Jlo, (float *)Jf, hf, jexp);
    else if (p.vtype == ISING_F32)
        hipLaunchKernelGGL(k_dense_split<float>, dim3(blocks), dim3(256), 0, s, p, Mp, Kp, form,
                           (unsigned short *)Jhi, (unsigned short *)Jlo, (float *)Jf, hf, jexp);
    else
        hipLaunchKernelGGL(k_dense_split<double>, dim3(blocks), dim3(256), 0, s, p, Mp, Kp, form,
                           (unsigned short *)Jhi, (unsigned short *)Jlo, (float *)Jf, hf, jexp);
    return hipGetLastError();
}

// host side of one problem's descriptor
static DenseDesc make_desc(const DenseRun &d) {
    DenseDesc a{};
    a.n = d.n;
    a.R = d.R;
    a.Mp = d.Mp;
    a.Kp = d.Kp;
    a.opt = d.opt;
    a.mtiles = d.Mp / BM;
    a.lr = (float)d.lr;
    a.mu = (float)d.mu;
    a.b1 = (float)d.b1;
    a.b2 = (float)d.b2;
    a.eps = (float)d.eps;
    a.omb1 = (float)(1.0 - d.b1);
    a.omb2 = (float)(1.0 - d.b2);
    a.t0 = d.t0;
    a.bias = d.bias;
    a.Jhi = (const unsigned short *)d.Jhi;
    a.Jlo = (const unsigned short *)d.Jlo;
    a.Jf = (const float *)d.Jf;
    a.h = d.h;
    const size_t sbytes = dense_vertex_bytes(d.form);
    a.jscale = d.form == DF_FP8 ? d.jscale : 1.f;
    a.jpow = int8_form(d.form) ? (const float *)((const char *)d.jsc + 16) : nullptr;
    a.S0 = (char *)d.S;
    a.S1 = (char *)d.S + (size_t)d.R * d.Kp * sbytes;
    a.S2 = (char *)d.S + (size_t)2 * d.R * d.Kp * sbytes;
    a.theta = d.theta;
    a.m = d.m;
    a.v = d.v;
    a.Epart = d.Epart;
    a.Lpart = d.Lpart;
    a.e_best = d.e_best;
    a.best_step = d.best_step;
    a.s_best = d.s_best;
    a.etrace = d.etrace;
    a.ltrace = d.ltrace;
    return a;
}

static size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

size_t dense_group_scratch_bytes(const DenseRun *const *runs, int count) {
    size_t tiles = 0, quads = 0;
    for (int k = 0; k < count; ++k) {
        tiles += (size_t)(runs[k]->Mp / BM) * ((runs[k]->R + tile_bn(runs[k]->form) - 1) / tile_bn(runs[k]->form));
        quads += (size_t)(runs[k]->R + 3) / 4;
    }
    return align16(count * sizeof(DenseDesc)) + tiles * sizeof(int4) + quads * sizeof(int2) + 64;
}

hipError_t dense_group_upload(const DenseRun *const *runs, int count, void *scratch, hipStream_t s,
                              DenseGroupShape *shape) {
    if (count <= 0) return hipErrorInvalidValue;
    const int form = runs[0]->form;
    std::vector<DenseDesc> descs;
    std::vector<int2> quads;
    // XCD-aware tile order.  Workgroups go to the 8 XCDs round-robin by index, each XCD with
    // its own L2, and a step's tiles run together.  Each problem's tiles are split into a
    // 2 x 4 grid of blocks (halves of the row tiles by quarters of the replica tiles), one
    // block per XCD: an XCD then reads half of J and a quarter of the vertex operand, where
    // a row-tile-fastest order would have every XCD read all of the vertex operand.  Only the
    // order of independent tiles changes.
    constexpr int kXcds = 8, kRowGroups = 2, kColGroups = kXcds / kRowGroups;
    std::vector<int4> per_xcd[kXcds];
    for (int k = 0; k < count; ++k) {
        const DenseRun &d = *runs[k];
        if (d.form != form || d.Mp % BM || d.Kp % (byte_form(d.form) ? 2 * KCB : KCB) || d.Mp < d.n || d.Kp < d.n)
            return hipErrorInvalidValue;
        if (int8_form(d.form) && !d.jsc) return hipErrorInvalidValue;
        if (d.opt == ISING_OPT_ADAM && !d.bias) return hipErrorInvalidValue;
        descs.push_back(make_desc(d));
        const int MT = d.Mp / BM, NT = (d.R + tile_bn(form) - 1) / tile_bn(form);
        for (int nt = 0; nt < NT; ++nt)
            for (int mt = 0; mt < MT; ++mt) {
                const int x = (mt * kRowGroups / MT) * kColGroups + nt * kColGroups / NT;
                per_xcd[x].push_back(make_int4(k, mt, nt, 0));
            }
        for (int q = 0; q < (d.R + 3) / 4; ++q) quads.push_back(make_int2(k, q));
    }
    // position p goes to XCD p % 8: deal the blocks' tiles out in that order (uneven blocks
    // leave a tail in another order, which only costs locality)
    std::vector<int4> tiles;
    size_t next[kXcds] = {};
    for (bool more = true; more;) {
        more = false;
        for (int x = 0; x < kXcds; ++x)
            if (next[x] < per_xcd[x].size()) {
                tiles.push_back(per_xcd[x][next[x]++]);
                more = true;
            }
    }
    char *p = (char *)scratch;
    DenseDesc *dd = (DenseDesc *)p;
    int4 *dt = (int4 *)(p + align16(descs.size() * sizeof(DenseDesc)));
    int2 *dq = (int2 *)((char *)dt + tiles.size() * sizeof(int4));
    hipError_t e = hipMemcpyAsync(dd, descs.data(), descs.size() * sizeof(DenseDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dq, quads.data(), quads.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    // the copies read the host vectors above: let them finish before the vectors go away
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    shape->form = form;
    shape->descs = count;
    shape->tiles = (int)tiles.size();
    shape->quads = (int)quads.size();
    return hipSuccess;
}

hipError_t dense_group_launch(const DenseGroupShape &shape, void *scratch, int steps, hipStream_t s) {
    char *p = (char *)scratch;
    // the layout of dense_group_upload: descriptors, then tiles, then quads
    const DenseDesc *dd = (const DenseDesc *)p;
    const int4 *dt = (const int4 *)(p + align16((size_t)shape.descs * sizeof(DenseDesc)));
    const int2 *dq = (const int2 *)((const char *)dt + (size_t)shape.tiles * sizeof(int4));
    for (int t = 1; t <= steps; ++t) {
        const dim3 blk(tile_threads(shape.form));
        if (shape.form == DF_FP32) hipLaunchKernelGGL(k_dense_step<DF_FP32>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
        else if (shape.form == DF_BF16X2) hipLaunchKernelGGL(k_dense_step<DF_BF16X2>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
        else if (shape.form == DF_FP8) hipLaunchKernelGGL(k_dense_step<DF_FP8>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
        else if (shape.form == DF_I8X3) hipLaunchKernelGGL(k_dense_step<DF_I8X3>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
        else if (shape.form == DF_I8X2) hipLaunchKernelGGL(k_dense_step<DF_I8X2>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
        else if (shape.form == DF_I8X1) hipLaunchKernelGGL(k_dense_step<DF_I8X1>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
        else hipLaunchKernelGGL(k_dense_step<DF_BF16>, dim3(shape.tiles), blk, 0, s, dd, dt, t);
    }
    // the last step's best-vertex bookkeeping (earlier steps are kept inside the next step)
    if (steps > 0) hipLaunchKernelGGL(k_dense_best, dim3(shape.quads), dim3(256), 0, s, dd, dq, steps, shape.form);
    return hipGetLastError();
}

hipError_t launch_dense_group(const DenseRun *const *runs, int count, int steps, void *scratch, hipStream_t s) {
    if (count <= 0 || steps <= 0) return hipSuccess;
    DenseGroupShape shape;
    hipError_t e = dense_group_upload(runs, count, scratch, s, &shape);
    if (e != hipSuccess) return e;
    return dense_group_launch(shape, scratch, steps, s);
}

hipError_t launch_dense_init(const DenseRun &d, hipStream_t s) {
    // (re)derive the vertex buffer from theta at every chunk; initialise the state at t0 = 0
    const size_t sbytes = dense_vertex_bytes(d.form);
    char *S0 = (char *)d.S;
    char *S1 = S0 + (size_t)d.R * d.Kp * sbytes;
    char *S2 = S1 + (size_t)d.R * d.Kp * sbytes;
    const int64_t total = (int64_t)d.R * d.Kp;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_dense_init, dim3(blocks), dim3(256), 0, s, d.n, d.R, d.Kp, d.form,
                       d.t0 == 0 ? d.init_mode : 0, d.seed, (const float *)d.uniform, d.theta, d.m, d.v,
                       (void *)S0, (void *)S1, (void *)S2, d.e_best, d.best_step, d.s_best);
    return hipGetLastError();
}

hipError_t launch_dense_run(const DenseRun &d, void *scratch, hipStream_t s) {
    hipError_t e = launch_dense_init(d, s);
    if (e != hipSuccess) return e;
    const DenseRun *one = &d;
    return launch_dense_group(&one, 1, d.steps, scratch, s);
}

}  // namespace ising
