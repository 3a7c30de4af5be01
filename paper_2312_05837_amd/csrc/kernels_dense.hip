// Domain selection for dense couplings on the matrix cores (paper Sec. III-B).
//
// One launch per step: Y = J S~ (rows = spins, columns = replicas) on MFMA,
// then the step's elementwise update fused into the tile epilogue while the
// accumulators are still in registers:
//   E_r partial += s (y + h),  L_r partial += sin(theta) (y - mu s + h),
//   GD / ADAM update of theta, wrap, next vertex S~' = sgn(sin theta') written
//   as the next step's B operand.
// A small second kernel combines the per-row-tile energy partials in a fixed
// order, keeps each replica's best energy and copies the vertex of an
// improvement.
//
// Forms of the coupling product (the iterates are FP32 in all of them):
//   DF_FP32   J and S~ in FP32, v_mfma_f32_32x32x2_f32
//   DF_BF16X2 J = J_hi + J_lo, both BF16 (J_hi = bf16(J), J_lo = bf16(J - J_hi)),
//             S~ = +-1 exact in BF16, two v_mfma_f32_32x32x16_bf16 per k-step
//             into the same FP32 accumulators
//   DF_BF16   J_hi only
// Tile: 128 spins x 128 replicas per workgroup of four wavefronts (2 x 2, each
// 64 x 64 = 2 x 2 MFMA blocks of 32 x 32), K staged through LDS in chunks of 32.
// Operand layouts: J padded row-major [Mp][Kp]; S~ replica-major [R][Kp]
// (each replica's spins contiguous), so both MFMA operands are K-contiguous.
// State theta, m, v, s_best: replica-major [R][n].
#include "internal.hpp"

namespace ising {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128, KC = 32;
constexpr int AST = KC + 8;   // LDS row stride (bf16 elements) of the A and B chunks
constexpr int FST = KC + 1;   // LDS row stride (floats) for the FP32 form

__device__ inline unsigned short bf16_bits(float x) {
    // round to nearest even
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ inline float bf16_to_f(unsigned short b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

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

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---- operand preparation ----------------------------------------------------

template <typename V>
__global__ void k_dense_split(DevProblem p, int Mp, int Kp, int form, unsigned short *Jhi, unsigned short *Jlo,
                              float *Jf, float *hf) {
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
        } else {
            const float vf = (float)v;
            const unsigned short hi = bf16_bits(vf);
            Jhi[q] = hi;
            if (form == DF_BF16X2) Jlo[q] = bf16_bits((float)(v - (double)bf16_to_f(hi)));
        }
    }
}

// theta_0 = asin(U), m = v = 0, S~_1 = sgn(sin theta_0) (padding zero), e_best = +inf
__global__ void k_dense_init(int n, int R, int Kp, int form, int init_mode, uint64_t seed, const float *uniform,
                             float *theta, float *m, float *v, void *S, void *S_other, double *e_best,
                             int32_t *best_step, int8_t *s_best) {
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
            ((float *)S_other)[q] = 0.f;  // the other buffer's padding must be zero too
        } else {
            ((unsigned short *)S)[q] = bf16_bits(s);
            ((unsigned short *)S_other)[q] = 0;
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

struct DenseStepArgs {
    int n, R, Mp, Kp, opt;
    float lr, mu, b1, b2, eps, omb1, omb2, ib1, ib2;
    const unsigned short *Jhi, *Jlo;
    const float *Jf;
    const float *h;
    const void *S_in;
    void *S_out;
    float *theta, *m, *v;
    float *Epart, *Lpart;  // [Mtiles][R]
};

template <int FORM>
__global__ __launch_bounds__(256) void k_dense_step(const DenseStepArgs a) {
    __shared__ __align__(16) unsigned char lds[FORM == DF_FP32 ? (BM + BN) * FST * 4 : (2 * BM + BN) * AST * 2];
    __shared__ float red_e[2][BN], red_l[2][BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int mt = blockIdx.x, nt = blockIdx.y;
    const int row0 = mt * BM, col0 = nt * BN;
    f32x16 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x16{};

    for (int k0 = 0; k0 < a.Kp; k0 += KC) {
        if constexpr (FORM == DF_FP32) {
            float *As = (float *)lds;
            float *Bs = As + BM * FST;
            // A: 128 rows x 32 floats; each thread loads 16 floats (4 x float4)
            for (int q = tid; q < BM * KC / 4; q += 256) {
                const int r = q / (KC / 4), c4 = (q % (KC / 4)) * 4;
                const float4 x = *(const float4 *)(a.Jf + (size_t)(row0 + r) * a.Kp + k0 + c4);
                As[r * FST + c4] = x.x; As[r * FST + c4 + 1] = x.y; As[r * FST + c4 + 2] = x.z; As[r * FST + c4 + 3] = x.w;
            }
            for (int q = tid; q < BN * KC / 4; q += 256) {
                const int r = q / (KC / 4), c4 = (q % (KC / 4)) * 4;
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (col0 + r < a.R) x = *(const float4 *)((const float *)a.S_in + (size_t)(col0 + r) * a.Kp + k0 + c4);
                Bs[r * FST + c4] = x.x; Bs[r * FST + c4 + 1] = x.y; Bs[r * FST + c4 + 2] = x.z; Bs[r * FST + c4 + 3] = x.w;
            }
            __syncthreads();
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
            __syncthreads();
        } else {
            unsigned short *Ah = (unsigned short *)lds;
            unsigned short *Al = Ah + BM * AST;
            unsigned short *Bs = Al + BM * AST;
            // A chunk: 128 rows x 32 bf16 = 4 x 16 B per row; 512 vectors per operand
            for (int q = tid; q < BM * 4; q += 256) {
                const int r = q >> 2, c8 = (q & 3) * 8;
                *(u16x8 *)(Ah + r * AST + c8) = *(const u16x8 *)(a.Jhi + (size_t)(row0 + r) * a.Kp + k0 + c8);
                if (FORM == DF_BF16X2)
                    *(u16x8 *)(Al + r * AST + c8) = *(const u16x8 *)(a.Jlo + (size_t)(row0 + r) * a.Kp + k0 + c8);
            }
            for (int q = tid; q < BN * 4; q += 256) {
                const int r = q >> 2, c8 = (q & 3) * 8;
                u16x8 x = u16x8{};
                if (col0 + r < a.R)
                    x = *(const u16x8 *)((const unsigned short *)a.S_in + (size_t)(col0 + r) * a.Kp + k0 + c8);
                *(u16x8 *)(Bs + r * AST + c8) = x;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < KC; ks += 16) {
                const int kk = ks + 8 * (lane >> 5);
                bf16x8 ah[2], al[2], bv[2];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) {
                    const int r = wm * 64 + bi * 32 + (lane & 31);
                    ah[bi] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(Ah + r * AST + kk));
                    if (FORM == DF_BF16X2) al[bi] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(Al + r * AST + kk));
                }
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const int c = wn * 64 + bj * 32 + (lane & 31);
                    bv[bj] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(Bs + c * AST + kk));
                }
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) {
                        if (FORM == DF_BF16X2)
                            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bv[bj], acc[bi][bj], 0, 0, 0);
                        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bv[bj], acc[bi][bj], 0, 0, 0);
                    }
            }
            __syncthreads();
        }
    }

    // ---- fused epilogue: C block (bi, bj), lane l, element q ->
    //      row 64 wm + 32 bi + 8 (q / 4) + 4 (l / 32) + q % 4, column 64 wn + 32 bj + l % 32
    const bool adam = a.opt == ISING_OPT_ADAM;
    float Ecol[2] = {0.f, 0.f}, Lcol[2] = {0.f, 0.f};
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int r = col0 + wn * 64 + bj * 32 + (lane & 31);
        if (r >= a.R) continue;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = row0 + wm * 64 + bi * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                if (i >= a.n) continue;
                const size_t idx = (size_t)r * a.n + i;
                const float y = acc[bi][bj][q];
                const float th = a.theta[idx];
                float x, c;
                fsincos(th, &x, &c);
                const bool neg = x < 0.f;
                const float yh = y + (a.h ? a.h[i] : 0.f);
                Ecol[bj] += neg ? -yh : yh;
                const float tt = neg ? yh + a.mu : yh - a.mu;
                Lcol[bj] += x * tt;
                const float g = c * tt;
                float upd;
                if (adam) {
                    const float mo = a.b1 * a.m[idx] + a.omb1 * g;
                    const float ve = a.b2 * a.v[idx] + a.omb2 * (g * g);
                    a.m[idx] = mo;
                    a.v[idx] = ve;
                    upd = a.lr * (mo * a.ib1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(ve * a.ib2) + a.eps);
                } else {
                    upd = a.lr * g;
                }
                float tn = th - upd;
                const float kq = rintf(tn * 0.159154943091895336f);
                tn = tn - kq * 6.28318548202514648f;
                tn = tn - kq * -1.7484555314695172e-07f;
                a.theta[idx] = tn;
                float xn, cn;
                fsincos(tn, &xn, &cn);
                const float sn = xn < 0.f ? -1.f : 1.f;
                if (FORM == DF_FP32) ((float *)a.S_out)[(size_t)r * a.Kp + i] = sn;
                else ((unsigned short *)a.S_out)[(size_t)r * a.Kp + i] = bf16_bits(sn);
            }
        }
    }
    // combine the two lane halves (rows +4) of each column, then the two row-waves
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        Ecol[bj] += __shfl_xor(Ecol[bj], 32);
        Lcol[bj] += __shfl_xor(Lcol[bj], 32);
    }
    if (lane < 32) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            red_e[wm][wn * 64 + bj * 32 + lane] = Ecol[bj];
            red_l[wm][wn * 64 + bj * 32 + lane] = Lcol[bj];
        }
    }
    __syncthreads();
    if (tid < BN && col0 + tid < a.R) {
        a.Epart[(size_t)mt * a.R + col0 + tid] = red_e[0][tid] + red_e[1][tid];
        if (a.Lpart) a.Lpart[(size_t)mt * a.R + col0 + tid] = red_l[0][tid] + red_l[1][tid];
    }
}

// one wavefront per replica: E_t from the row-tile partials (ascending), best-vertex update
__global__ __launch_bounds__(256) void k_dense_best(int n, int R, int Kp, int mtiles, int form, int tglobal,
                                                    const float *Epart, const float *Lpart, const void *S_t,
                                                    double *e_best, int32_t *best_step, int8_t *s_best,
                                                    double *etrace, double *ltrace) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= R) return;
    float E = 0.f, L = 0.f;
    for (int t = 0; t < mtiles; ++t) {
        E += Epart[(size_t)t * R + r];
        if (Lpart) L += Lpart[(size_t)t * R + r];
    }
    const bool imp = (double)E < e_best[r];
    if (imp) {
        for (int i = lane; i < n; i += 64) {
            const float s = form == DF_FP32 ? ((const float *)S_t)[(size_t)r * Kp + i]
                                            : bf16_to_f(((const unsigned short *)S_t)[(size_t)r * Kp + i]);
            s_best[(size_t)r * n + i] = s < 0.f ? (int8_t)-1 : (int8_t)1;
        }
    }
    if (lane == 0) {
        if (imp) {
            e_best[r] = (double)E;
            best_step[r] = tglobal;
        }
        if (etrace) etrace[r] = (double)E;
        if (ltrace) ltrace[r] = (double)L;
    }
}

}  // namespace

hipError_t launch_dense_prepare(const DevProblem &p, int form, int Mp, int Kp, void *Jhi, void *Jlo, void *Jf,
                                float *hf, hipStream_t s) {
    const int64_t total = (int64_t)Mp * Kp;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    if (p.vtype == ISING_I32)
        hipLaunchKernelGGL(k_dense_split<int32_t>, dim3(blocks), dim3(256), 0, s, p, Mp, Kp, form,
                           (unsigned short *)Jhi, (unsigned short *)Jlo, (float *)Jf, hf);
    else if (p.vtype == ISING_F32)
        hipLaunchKernelGGL(k_dense_split<float>, dim3(blocks), dim3(256), 0, s, p, Mp, Kp, form,
                           (unsigned short *)Jhi, (unsigned short *)Jlo, (float *)Jf, hf);
    else
        hipLaunchKernelGGL(k_dense_split<double>, dim3(blocks), dim3(256), 0, s, p, Mp, Kp, form,
                           (unsigned short *)Jhi, (unsigned short *)Jlo, (float *)Jf, hf);
    return hipGetLastError();
}

hipError_t launch_dense_run(const DenseRun &d, hipStream_t s) {
    const int mtiles = d.Mp / BM, ntiles = (d.R + BN - 1) / BN;
    if (d.Mp % BM || d.Kp % KC || d.Mp < d.n || d.Kp < d.n) return hipErrorInvalidValue;
    const size_t sbytes = d.form == DF_FP32 ? 4 : 2;
    char *S0 = (char *)d.S;
    char *S1 = S0 + (size_t)d.R * d.Kp * sbytes;
    {  // (re)derive the vertex buffer from theta at every call; initialise the state at t0 = 0
        const int64_t total = (int64_t)d.R * d.Kp;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
        hipLaunchKernelGGL(k_dense_init, dim3(blocks), dim3(256), 0, s, d.n, d.R, d.Kp, d.form,
                           d.t0 == 0 ? d.init_mode : 0, d.seed, (const float *)d.uniform, d.theta, d.m, d.v,
                           (void *)S0, (void *)S1, d.e_best, d.best_step, d.s_best);
    }
    DenseStepArgs a;
    a.n = d.n;
    a.R = d.R;
    a.Mp = d.Mp;
    a.Kp = d.Kp;
    a.opt = d.opt;
    a.lr = (float)d.lr;
    a.mu = (float)d.mu;
    a.b1 = (float)d.b1;
    a.b2 = (float)d.b2;
    a.eps = (float)d.eps;
    a.omb1 = (float)(1.0 - d.b1);
    a.omb2 = (float)(1.0 - d.b2);
    a.Jhi = (const unsigned short *)d.Jhi;
    a.Jlo = (const unsigned short *)d.Jlo;
    a.Jf = (const float *)d.Jf;
    a.h = d.h;
    a.theta = d.theta;
    a.m = d.m;
    a.v = d.v;
    a.Epart = d.Epart;
    a.Lpart = d.ltrace ? d.Lpart : nullptr;
    for (int t = 1; t <= d.steps; ++t) {
        const int tg = d.t0 + t;
        a.ib1 = (float)(1.0 / -std::expm1(tg * std::log(d.b1)));
        a.ib2 = (float)(1.0 / -std::expm1(tg * std::log(d.b2)));
        // S buffer k % 2 holds the vertex of step t0 + k + 1 counted from the last (re)initialisation
        const int cur = (t - 1) & 1;
        a.S_in = cur ? S1 : S0;
        a.S_out = cur ? S0 : S1;
        dim3 grid(mtiles, ntiles);
        if (d.form == DF_FP32) hipLaunchKernelGGL(k_dense_step<DF_FP32>, grid, dim3(256), 0, s, a);
        else if (d.form == DF_BF16X2) hipLaunchKernelGGL(k_dense_step<DF_BF16X2>, grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_dense_step<DF_BF16>, grid, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_dense_best, dim3((d.R + 3) / 4), dim3(256), 0, s, d.n, d.R, d.Kp, mtiles, d.form, tg,
                           (const float *)d.Epart, (const float *)a.Lpart, a.S_in, d.e_best, d.best_step, d.s_best,
                           d.etrace ? d.etrace + (size_t)(t - 1) * d.R : nullptr,
                           d.ltrace ? d.ltrace + (size_t)(t - 1) * d.R : nullptr);
    }
    return hipGetLastError();
}

}  // namespace ising
