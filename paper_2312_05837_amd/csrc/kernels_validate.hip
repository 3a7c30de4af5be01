// Ingest checks of a problem on the device: symmetry, zero diagonal, CSR
// structure, finiteness, maximum degree, common coupling magnitude and
// integrality.  One pass over J.
#include "internal.hpp"

namespace ising {

template <typename V>
__device__ inline double as_double(const void *p, int64_t k) {
    return (double)(((const V *)p)[k]);
}

__device__ inline double load_val(const void *p, int vtype, int64_t k) {
    if (vtype == ISING_I32) return as_double<int32_t>(p, k);
    if (vtype == ISING_F32) return as_double<float>(p, k);
    return as_double<double>(p, k);
}

__device__ inline bool is_integral(double x) { return x == rint(x) && fabs(x) < 9.0e15; }

// Combine one thread's findings over the workgroup and publish them with at most
// one atomic per flag and workgroup (every thread of the workgroup must call it).
__device__ void publish_flags(int bits, int deg, bool uni, bool integ, int32_t *flags, int maxabs = 0) {
    __shared__ int s_bits, s_deg, s_abs;
    if (threadIdx.x == 0) {
        s_bits = 0;
        s_deg = 0;
        s_abs = 0;
    }
    __syncthreads();
    if (bits) atomicOr(&s_bits, bits);
    if (deg > 0) atomicMax(&s_deg, deg);
    if (maxabs > 0) atomicMax(&s_abs, maxabs);
    const bool any_nonuni = __syncthreads_or(!uni);
    const bool any_nonint = __syncthreads_or(!integ);
    if (threadIdx.x == 0) {
        if (s_bits) atomicOr(&flags[0], s_bits);
        if (s_deg > 0) atomicMax(&flags[1], s_deg);
        if (s_abs > 0) atomicMax(&flags[4], s_abs);
        if (any_nonuni) atomicAnd(&flags[2], 0);
        if (any_nonint) atomicAnd(&flags[3], 0);
    }
}

// |a| as an int when a is integral and below 2^30 (0 otherwise): largest integer coupling magnitude
__device__ inline int int_magnitude(double a) {
    const double m = fabs(a);
    return (m == floor(m) && m < 1073741824.0) ? (int)m : 0;
}

// flags: [0] error bits, [1] max degree (atomicMax), [2] uniform magnitude (cleared on mismatch),
// [3] integral (cleared on a non-integral value)
// One 32 x 32 tile (bi, bj) with bi <= bj per workgroup: the tile and its mirror
// are read coalesced into LDS and compared element by element.
__global__ __launch_bounds__(256) void validate_dense(DevProblem p, double w0, int32_t *flags) {
    __shared__ double A[32][33], Bt[32][33];
    const int nt = (p.n + 31) / 32;
    // map the linear block index to an upper-triangular tile (bi <= bj)
    int b = blockIdx.x, bi = 0;
    while (b >= nt - bi) {
        b -= nt - bi;
        ++bi;
    }
    const int bj = bi + b;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int n = p.n;
    for (int yy = ty; yy < 32; yy += 8) {
        const int i = bi * 32 + yy, j = bj * 32 + tx;
        A[yy][tx] = (i < n && j < n) ? load_val(p.J, p.vtype, (int64_t)i * n + j) : 0.0;
        const int i2 = bj * 32 + yy, j2 = bi * 32 + tx;
        Bt[yy][tx] = (i2 < n && j2 < n) ? load_val(p.J, p.vtype, (int64_t)i2 * n + j2) : 0.0;
    }
    __syncthreads();
    int bits = 0, mabs = 0;
    bool uni = true, integ = true;
    for (int yy = ty; yy < 32; yy += 8) {
        const int i = bi * 32 + yy, j = bj * 32 + tx;
        if (i >= n || j >= n) continue;
        const double a = A[yy][tx];
        const double m = Bt[tx][yy];  // J[j][i]
        mabs = max(mabs, max(int_magnitude(a), int_magnitude(m)));
        if (!isfinite(a)) bits |= 8;
        if (i == j) {
            if (a != 0.0) bits |= 2;
        } else {
            if (a != m) bits |= 1;
            if (a != 0.0) {
                if (fabs(a) != w0) uni = false;
                if (!is_integral(a)) integ = false;
            }
            if (bi != bj) {  // the mirror tile's element is checked here too
                if (!isfinite(m)) bits |= 8;
                if (m != 0.0) {
                    if (fabs(m) != w0) uni = false;
                    if (!is_integral(m)) integ = false;
                }
            }
        }
    }
    publish_flags(bits, 0, uni, integ, flags, mabs);
}

__global__ void dense_degree(DevProblem p, int32_t *flags) {
    // one wave per row: count nonzeros
    const int n = p.n;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    int c = 0;
    if (row < n)
        for (int j = lane; j < n; j += 64)
            c += load_val(p.J, p.vtype, (int64_t)row * n + j) != 0.0;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    publish_flags(0, lane == 0 ? c : 0, true, true, flags);
}

__global__ void validate_csr(DevProblem p, double w0, int32_t *flags) {
    const int n = p.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int bits = 0, mabs = 0;
    bool uni = true, integ = true;
    int rs = 0, re = 0;
    if (i < n) {
        rs = p.row_ptr[i];
        re = p.row_ptr[i + 1];
        if (rs < 0 || re < rs || re > p.nnz) {
            bits = 4;
            rs = re = 0;
        }
    }
    int prev = -1;
    for (int k = rs; k < re; ++k) {
        const int j = p.col[k];
        if (j < 0 || j >= n || j <= prev) {
            bits |= 4;
            break;
        }
        prev = j;
        if (j == i) bits |= 2;
        const double a = load_val(p.val, p.vtype, k);
        if (!isfinite(a)) bits |= 8;
        mabs = max(mabs, int_magnitude(a));
        if (fabs(a) != w0) uni = false;
        if (!is_integral(a)) integ = false;
        // symmetric partner: binary search row j for column i
        const int js = p.row_ptr[j], je = p.row_ptr[j + 1];
        if (js < 0 || je < js || je > p.nnz) {
            bits |= 4;
            break;
        }
        int lo = js, hi = je - 1, found = -1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int c = p.col[mid];
            if (c == i) {
                found = mid;
                break;
            }
            if (c < i) lo = mid + 1;
            else hi = mid - 1;
        }
        if (found < 0 || load_val(p.val, p.vtype, found) != a) bits |= 1;
    }
    publish_flags(bits, re - rs, uni, integ, flags, mabs);
}

__global__ void validate_h(DevProblem p, int32_t *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int bits = 0;
    bool integ = true;
    if (i < p.n && p.h != nullptr) {
        const double a = load_val(p.h, p.vtype, i);
        if (!isfinite(a)) bits = 8;
        if (!is_integral(a)) integ = false;
    }
    publish_flags(bits, 0, true, integ, flags);
}

__global__ void first_magnitude(DevProblem p, double *w) {
    // magnitude of the first nonzero coupling (row-major order); 1.0 if none
    if (threadIdx.x != 0) return;
    double r = 1.0;
    if (p.format == ISING_CSR) {
        if (p.nnz > 0) r = fabs(load_val(p.val, p.vtype, 0));
    } else {
        const int64_t total = (int64_t)p.n * p.n;
        for (int64_t k = 0; k < total; ++k) {
            const double a = load_val(p.J, p.vtype, k);
            if (a != 0.0) {
                r = fabs(a);
                break;
            }
        }
    }
    *w = r;
}

hipError_t launch_first_magnitude(const DevProblem &p, double *w, hipStream_t s) {
    hipLaunchKernelGGL(first_magnitude, dim3(1), dim3(64), 0, s, p, w);
    return hipGetLastError();
}

__global__ void init_flags(int32_t *flags) {
    if (threadIdx.x == 0) {
        flags[0] = 0;
        flags[1] = 0;
        flags[2] = 1;
        flags[3] = 1;
        flags[4] = 0;
    }
}

hipError_t launch_validate_with(const DevProblem &p, double w0, int32_t *flags, hipStream_t s) {
    hipLaunchKernelGGL(init_flags, dim3(1), dim3(64), 0, s, flags);
    if (p.format == ISING_DENSE) {
        const int64_t nt = (p.n + 31) / 32;
        hipLaunchKernelGGL(validate_dense, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, p, w0, flags);
        hipLaunchKernelGGL(dense_degree, dim3((p.n + 3) / 4), dim3(256), 0, s, p, flags);
    } else {
        hipLaunchKernelGGL(validate_csr, dim3((p.n + 255) / 256), dim3(256), 0, s, p, w0, flags);
    }
    hipLaunchKernelGGL(validate_h, dim3((p.n + 255) / 256), dim3(256), 0, s, p, flags);
    return hipGetLastError();
}

hipError_t launch_validate(const DevProblem &p, int32_t *flags, double *wdev, hipStream_t s) {
    // the common magnitude candidate is needed on the host (ingest, not the hot loop)
    hipLaunchKernelGGL(first_magnitude, dim3(1), dim3(64), 0, s, p, wdev);
    double w0 = 1.0;
    hipError_t e = hipMemcpyAsync(&w0, wdev, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    return launch_validate_with(p, w0, flags, s);
}

}  // namespace ising
