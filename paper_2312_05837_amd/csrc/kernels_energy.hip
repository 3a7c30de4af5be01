// Exact energy E(s) = s^T J s + h^T s (paper, Sec. II, scalar energy form) for a
// block of spin vectors.  Integer problems accumulate in int64 (exact, order
// free).  Real problems accumulate in FP64: one wavefront per row (64 strided
// partials over the row's stored positions, xor butterfly), the four rows of a
// block in index order, blocks in ascending order -- reproducible run to run.
#include <mutex>

#include "internal.hpp"

namespace ising {

namespace {

constexpr int EB = 4;  // rows per block (one wavefront each)

template <typename V, typename Acc>
__global__ __launch_bounds__(256) void energy_rows(DevProblem p, const int8_t *spins, Acc *partial) {
    __shared__ Acc red[4];
    const int n = p.n;
    const int r = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * EB + wv;
    const int8_t *s = spins + (size_t)r * n;
    Acc y = 0;
    if (i < n) {
        if (p.format == ISING_DENSE) {
            const V *row = (const V *)p.J + (size_t)i * n;
            for (int j = lane; j < n; j += 64) y += (Acc)row[j] * (Acc)s[j];
        } else {
            const int rs = p.row_ptr[i], len = p.row_ptr[i + 1] - rs;
            const V *val = (const V *)p.val + rs;
            const int32_t *col = p.col + rs;
            for (int q = lane; q < len; q += 64) y += (Acc)val[q] * (Acc)s[col[q]];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d);
    if (lane == 0) {
        Acc term = 0;
        if (i < n) {
            const Acc hi = p.h ? (Acc)((const V *)p.h)[i] : (Acc)0;
            term = (Acc)s[i] * (y + hi);
        }
        red[wv] = term;
    }
    __syncthreads();
    if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename Acc>
__global__ void energy_finish(const Acc *partial, int nblocks, int count, double *E_out,
                              int64_t *E_int_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    Acc t = 0;
    for (int b = 0; b < nblocks; ++b) t += partial[(size_t)r * nblocks + b];
    if (E_out) E_out[r] = (double)t;
    if (E_int_out) E_int_out[r] = (int64_t)t;
}

// Scratch for the energy partials of the entry point that allocates nothing: one array per
// GPU the library runs on, held until the process ends.  Host code never uses this name as an
// address (on the host it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kEnergyScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t energy_partial_bytes(int32_t n, int32_t count) {
    return (size_t)count * ((n + EB - 1) / EB) * 8;
}

hipError_t energy_scratch_address(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[device] = p;
    }
    *ptr = scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_energy(const DevProblem &p, const int8_t *spins, int32_t count, void *partial,
                         double *E_out, int64_t *E_int_out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int nb = (p.n + EB - 1) / EB;
    dim3 grid(nb, count);
    const int fb = (count + 63) / 64;
    if (p.vtype == ISING_I32) {
        hipLaunchKernelGGL((energy_rows<int32_t, int64_t>), grid, dim3(256), 0, s, p, spins,
                           (int64_t *)partial);
        hipLaunchKernelGGL((energy_finish<int64_t>), dim3(fb), dim3(64), 0, s, (const int64_t *)partial,
                           nb, count, E_out, E_int_out);
    } else if (p.vtype == ISING_F32) {
        hipLaunchKernelGGL((energy_rows<float, double>), grid, dim3(256), 0, s, p, spins,
                           (double *)partial);
        hipLaunchKernelGGL((energy_finish<double>), dim3(fb), dim3(64), 0, s, (const double *)partial,
                           nb, count, E_out, (int64_t *)nullptr);
    } else {
        hipLaunchKernelGGL((energy_rows<double, double>), grid, dim3(256), 0, s, p, spins,
                           (double *)partial);
        hipLaunchKernelGGL((energy_finish<double>), dim3(fb), dim3(64), 0, s, (const double *)partial,
                           nb, count, E_out, (int64_t *)nullptr);
    }
    return hipGetLastError();
}

}  // namespace ising
