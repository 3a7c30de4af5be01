// Pruning (paper Sec. III-A, Algorithm 1) and retrieval (Fig. 1c) on the device.
//
// One round, on the active set A:
//   rowsum_D : a_i = sum_{j in A} |J_ij| per row (one wavefront per row: 64
//              strided partials over the row's stored positions, combined by an
//              xor butterfly 32,16,8,4,2,1); D = {i in A : |h_i| > 2 a_i};
//              s_i = -sgn(h_i)  (determined-spin rule).
//   fold_D   : h_j += sum_{i in D} 2 J_ji s_i for j in A \ D;
//              C gets h_i s_i + sum_{j in D} J_ij s_i s_j per i in D.
//   degree   : deg_k over A \ D; candidate if deg_k = 1 and 2|J_k,n(k)| >= |h_k|.
//   select_S : of a mutual candidate pair only the larger index is taken.
//   fold_S   : h_i -= sum_{k in S, n(k) = i} sgn(J_ik) h_k;
//              C gets -2|J_k,n(k)| per k in S  (semi-determined-spin rule).
// Every per-row sum runs on one wavefront in the same fixed order as the row
// sums (64 strided partials, xor butterfly), with coalesced reads of the row.
// Integer problems work in int64 (exact); real problems in FP64.
//
// Rounds are enqueued ahead of the host's knowledge of whether they are needed:
// the round that removes nothing sets a done flag (counts[4]) and counts the
// rounds executed (counts[5]); every kernel of a later round sees the flag and
// returns at once, so the host reads the counters once per batch of rounds.
#include "internal.hpp"

namespace ising {

namespace {

template <typename W>
__device__ inline W wabs(W x) { return x < 0 ? -x : x; }

template <typename W>
__device__ inline int wsgn(W x) { return x > 0 ? 1 : (x < 0 ? -1 : 0); }

template <typename V, typename W>
__global__ void k_init(DevProblem p, PruneWork w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *(W *)w.C = 0;
        w.counts[0] = w.counts[1] = 0;
        w.counts[2] = p.n;
        w.counts[3] = 0;
        w.counts[4] = 0;
        w.counts[5] = 0;
    }
    if (i >= p.n) return;
    w.active[i] = 1;
    w.isD[i] = w.isS[i] = w.cand[i] = 0;
    w.kind[i] = 0;
    w.fixed[i] = 0;
    w.sigma[i] = 0;
    w.round_of[i] = -1;
    w.partner[i] = -1;
    w.nb[i] = -1;
    ((W *)w.h)[i] = p.h ? (W)((const V *)p.h)[i] : (W)0;
}

__global__ void k_round_begin(int32_t *counts) {
    if (threadIdx.x == 0 && !counts[4]) counts[0] = counts[1] = 0;
}

// after a round: count it, and set the done flag if it removed nothing
__global__ void k_round_end(int32_t *counts) {
    if (threadIdx.x == 0 && !counts[4]) {
        counts[5] += 1;
        if (counts[0] == 0 && counts[1] == 0) counts[4] = 1;
    }
}

// one wavefront per row
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_rowsum_D(DevProblem p, PruneWork w) {
    if (w.counts[4]) return;  // an earlier round removed nothing
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= p.n) return;
    if (!w.active[i]) {
        if (lane == 0) w.isD[i] = 0;
        return;
    }
    W acc = 0;
    if (p.format == ISING_DENSE) {
        const V *row = (const V *)p.J + (size_t)i * p.n;
        for (int j = lane; j < p.n; j += 64)
            if (w.active[j]) acc = acc + wabs((W)row[j]);
    } else {
        const int rs = p.row_ptr[i], len = p.row_ptr[i + 1] - rs;
        const V *val = (const V *)p.val + rs;
        const int32_t *col = p.col + rs;
        for (int q = lane; q < len; q += 64)
            if (w.active[col[q]]) acc = acc + wabs((W)val[q]);
    }
    for (int d = 32; d >= 1; d >>= 1) acc = acc + __shfl_xor(acc, d);
    if (lane == 0) {
        const W hi = ((const W *)w.h)[i];
        const bool d = wabs(hi) > 2 * acc;
        w.isD[i] = d;
        if (d) {
            w.fixed[i] = (int8_t)(-wsgn(hi));
            atomicAdd(&w.counts[0], 1);
        }
    }
}

// visit the entries of row i assigned to this lane (positions lane, lane + 64, ...)
template <typename V, typename F>
__device__ inline void lane_entries(const DevProblem &p, int i, int lane, F &&f) {
    if (p.format == ISING_DENSE) {
        const V *row = (const V *)p.J + (size_t)i * p.n;
        for (int j = lane; j < p.n; j += 64) f(j, row[j]);
    } else {
        const int rs = p.row_ptr[i], len = p.row_ptr[i + 1] - rs;
        const V *val = (const V *)p.val + rs;
        const int32_t *col = p.col + rs;
        for (int q = lane; q < len; q += 64) f(col[q], val[q]);
    }
}

template <typename W>
__device__ inline W wave_sum_fixed(W acc) {
    for (int d = 32; d >= 1; d >>= 1) acc = acc + __shfl_xor(acc, d);
    return acc;
}

// one wavefront per row j
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_fold_D(DevProblem p, PruneWork w, int round) {
    if (w.counts[4]) return;  // an earlier round removed nothing
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= p.n) return;
    W *h = (W *)w.h;
    W *cp = (W *)w.cpart;
    if (!w.active[j]) {
        if (lane == 0) cp[j] = 0;
        return;
    }
    const bool dj = w.isD[j];
    const W sj = dj ? (W)w.fixed[j] : (W)0;
    W acc = 0;
    lane_entries<V>(p, j, lane, [&](int i, V v) {
        if (w.isD[i]) {
            const W si = (W)w.fixed[i];
            acc = acc + (dj ? (W)v * sj * si : 2 * (W)v * si);
        }
    });
    acc = wave_sum_fixed(acc);
    if (lane == 0) {
        if (dj) {
            cp[j] = h[j] * sj + acc;
            w.kind[j] = 1;
            w.round_of[j] = round;
            w.active[j] = 0;
        } else {
            cp[j] = 0;
            h[j] = h[j] + acc;
        }
    }
}

// one wavefront per row k: active degree and the unique neighbour
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_degree(DevProblem p, PruneWork w) {
    if (w.counts[4]) return;  // an earlier round removed nothing
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= p.n) return;
    if (!w.active[k]) {
        if (lane == 0) w.cand[k] = 0;
        return;
    }
    int deg = 0, nbj = -1;
    W jvv = 0;
    lane_entries<V>(p, k, lane, [&](int j, V v) {
        if (v != 0 && w.active[j]) {
            ++deg;
            nbj = j;
            jvv = (W)v;
        }
    });
    for (int d = 32; d >= 1; d >>= 1) deg += __shfl_xor(deg, d);
    if (deg == 1) {
        const uint64_t m = __ballot(nbj >= 0);
        const int src = __builtin_ctzll(m);
        nbj = __shfl(nbj, src);
        jvv = __shfl(jvv, src);
    }
    if (lane == 0) {
        w.cand[k] = 0;
        if (deg == 1 && 2 * wabs(jvv) >= wabs(((const W *)w.h)[k])) {
            w.cand[k] = 1;
            w.nb[k] = nbj;
            ((W *)w.jv)[k] = jvv;
        }
    }
}

__global__ void k_select_S(int n, PruneWork w) {
    if (w.counts[4]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    bool s = false;
    if (w.cand[k]) {
        const int i = w.nb[k];
        const bool mutual = w.cand[i] && w.nb[i] == k;
        s = !(mutual && k < i);
    }
    w.isS[k] = s;
}

// one wavefront per row i
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_fold_S(DevProblem p, PruneWork w, int round) {
    if (w.counts[4]) return;  // an earlier round removed nothing
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= p.n) return;
    W *h = (W *)w.h;
    W *cp = (W *)w.cpart;
    if (w.isS[i]) {
        if (lane == 0) {
            const W jvi = ((const W *)w.jv)[i];
            cp[i] = -2 * wabs(jvi);
            w.kind[i] = 2;
            w.round_of[i] = round;
            w.partner[i] = w.nb[i];
            w.sigma[i] = (int8_t)wsgn(jvi);
            w.active[i] = 0;
            atomicAdd(&w.counts[1], 1);
        }
        return;
    }
    if (!w.active[i]) {
        if (lane == 0) cp[i] = 0;
        return;
    }
    W acc = 0;
    lane_entries<V>(p, i, lane, [&](int k, V v) {
        if (v != 0 && w.isS[k] && w.nb[k] == i) acc = acc + (W)wsgn((W)v) * h[k];
    });
    acc = wave_sum_fixed(acc);
    if (lane == 0) {
        cp[i] = 0;
        h[i] = h[i] - acc;
    }
}

// C += sum_i cpart[i]: each of 1024 threads sums i = tid, tid + 1024, ... in
// ascending order, then a fixed shared-memory tree.
template <typename W>
__global__ __launch_bounds__(1024) void k_accumulate_C(int n, PruneWork w) {
    __shared__ W red[1024];
    if (w.counts[4]) return;  // uniform over the workgroup: read before any barrier
    const W *cp = (const W *)w.cpart;
    W acc = 0;
    for (int i = threadIdx.x; i < n; i += 1024) acc = acc + cp[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if (threadIdx.x < d) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *(W *)w.C = *(W *)w.C + red[0];
}

// exclusive scan of flags (int8 active) -> map, G, counts[2]
__global__ __launch_bounds__(1024) void k_compact_scan(int n, PruneWork w) {
    __shared__ int part[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int c = 0;
    for (int i = lo; i < hi; ++i) c += w.active[i] ? 1 : 0;
    part[threadIdx.x] = c;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partials
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int base = part[threadIdx.x] - c;
    for (int i = lo; i < hi; ++i) {
        if (w.active[i]) {
            w.map[i] = base;
            w.G[base] = i;
            ++base;
        } else {
            w.map[i] = -1;
        }
    }
    if (threadIdx.x == 1023) w.counts[2] = part[1023];
}

// exclusive scan of cnt[0..m) into out[0..m], out[m] = total, counts[3] = total
__global__ __launch_bounds__(1024) void k_scan_counts(int m, int32_t *out, int32_t *counts) {
    __shared__ int part[1024];
    const int per = (m + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(m, lo + per);
    int c = 0;
    for (int i = lo; i < hi; ++i) c += out[i];
    part[threadIdx.x] = c;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int base = part[threadIdx.x] - c;
    for (int i = lo; i < hi; ++i) {
        const int x = out[i];
        out[i] = base;
        base += x;
    }
    if (threadIdx.x == 1023) {
        out[m] = part[1023];
        counts[3] = part[1023];
    }
}

template <typename V, typename W, typename O>
__global__ void k_gather_dense(DevProblem p, PruneWork w, int nG, O *JG, O *hG) {
    const int64_t total = (int64_t)nG * nG;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(q / nG), b = (int)(q % nG);
        JG[q] = (O)((const V *)p.J)[(size_t)w.G[a] * p.n + w.G[b]];
    }
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < nG) hG[a] = (O)((const W *)w.h)[w.G[a]];
}

template <typename V>
__global__ void k_csr_count(DevProblem p, PruneWork w, int nG, int32_t *rp) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nG) return;
    const int i = w.G[a];
    const V *val = (const V *)p.val;
    int c = 0;
    for (int q = p.row_ptr[i]; q < p.row_ptr[i + 1]; ++q) c += (w.active[p.col[q]] && val[q] != 0) ? 1 : 0;
    rp[a] = c;
}

template <typename V, typename W, typename O>
__global__ void k_csr_fill(DevProblem p, PruneWork w, int nG, const int32_t *rp, int32_t *colG, O *valG,
                           O *hG) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nG) return;
    const int i = w.G[a];
    const V *val = (const V *)p.val;
    int pos = rp[a];
    for (int q = p.row_ptr[i]; q < p.row_ptr[i + 1]; ++q) {
        const int j = p.col[q];
        if (w.active[j] && val[q] != 0) {
            colG[pos] = w.map[j];
            valG[pos] = (O)val[q];
            ++pos;
        }
    }
    hG[a] = (O)((const W *)w.h)[i];
}

__global__ __launch_bounds__(1024) void k_unprune(PruneWork w, int n, int rounds, const int8_t *sG,
                                                  int8_t *s) {
    for (int i = threadIdx.x; i < n; i += 1024) s[i] = w.kind[i] == 0 ? sG[w.map[i]] : (int8_t)0;
    __syncthreads();
    for (int r = rounds - 1; r >= 0; --r) {
        for (int i = threadIdx.x; i < n; i += 1024) {
            if (w.round_of[i] != r) continue;
            if (w.kind[i] == 1) s[i] = w.fixed[i];
            else s[i] = (int8_t)(-w.sigma[i] * s[w.partner[i]]);
        }
        __syncthreads();
    }
}

__global__ void k_copy_record(PruneWork w, int n, int8_t *kind, int32_t *round_of, int8_t *fixed,
                              int32_t *partner, int8_t *sigma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (kind) kind[i] = w.kind[i];
    if (round_of) round_of[i] = w.round_of[i];
    if (fixed) fixed[i] = w.kind[i] == 1 ? w.fixed[i] : (int8_t)0;
    if (partner) partner[i] = w.partner[i];
    if (sigma) sigma[i] = w.sigma[i];
}

inline dim3 g1(int n) { return dim3((n + 255) / 256); }

template <typename V, typename W>
hipError_t round_impl(const DevProblem &p, const PruneWork &w, int32_t round, hipStream_t s) {
    hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(64), 0, s, w.counts);
    hipLaunchKernelGGL((k_rowsum_D<V, W>), dim3((p.n + 3) / 4), dim3(256), 0, s, p, w);
    hipLaunchKernelGGL((k_fold_D<V, W>), dim3((p.n + 3) / 4), dim3(256), 0, s, p, w, round);
    hipLaunchKernelGGL((k_accumulate_C<W>), dim3(1), dim3(1024), 0, s, p.n, w);
    hipLaunchKernelGGL((k_degree<V, W>), dim3((p.n + 3) / 4), dim3(256), 0, s, p, w);
    hipLaunchKernelGGL(k_select_S, g1(p.n), dim3(256), 0, s, p.n, w);
    hipLaunchKernelGGL((k_fold_S<V, W>), dim3((p.n + 3) / 4), dim3(256), 0, s, p, w, round);
    hipLaunchKernelGGL((k_accumulate_C<W>), dim3(1), dim3(1024), 0, s, p.n, w);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, s, w.counts);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_prune_init(const DevProblem &p, const PruneWork &w, hipStream_t s) {
    if (p.vtype == ISING_I32) hipLaunchKernelGGL((k_init<int32_t, int64_t>), g1(p.n), dim3(256), 0, s, p, w);
    else if (p.vtype == ISING_F32) hipLaunchKernelGGL((k_init<float, double>), g1(p.n), dim3(256), 0, s, p, w);
    else hipLaunchKernelGGL((k_init<double, double>), g1(p.n), dim3(256), 0, s, p, w);
    return hipGetLastError();
}

hipError_t launch_prune_round(const DevProblem &p, const PruneWork &w, int32_t round, hipStream_t s) {
    if (p.vtype == ISING_I32) return round_impl<int32_t, int64_t>(p, w, round, s);
    if (p.vtype == ISING_F32) return round_impl<float, double>(p, w, round, s);
    return round_impl<double, double>(p, w, round, s);
}

hipError_t launch_prune_compact_scan(const DevProblem &p, const PruneWork &w, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, p.n, w);
    return hipGetLastError();
}

hipError_t launch_prune_gather_dense(const DevProblem &p, const PruneWork &w, int32_t nG, void *JG,
                                     void *hG, hipStream_t s) {
    const int64_t total = (int64_t)nG * nG;
    const int blocks = (int)std::max<int64_t>(std::min<int64_t>((total + 255) / 256, 8192), (nG + 255) / 256);
    if (p.vtype == ISING_I32)
        hipLaunchKernelGGL((k_gather_dense<int32_t, int64_t, int32_t>), dim3(blocks), dim3(256), 0, s, p, w,
                           nG, (int32_t *)JG, (int32_t *)hG);
    else if (p.vtype == ISING_F32)
        hipLaunchKernelGGL((k_gather_dense<float, double, double>), dim3(blocks), dim3(256), 0, s, p, w, nG,
                           (double *)JG, (double *)hG);
    else
        hipLaunchKernelGGL((k_gather_dense<double, double, double>), dim3(blocks), dim3(256), 0, s, p, w, nG,
                           (double *)JG, (double *)hG);
    return hipGetLastError();
}

hipError_t launch_prune_csr_count(const DevProblem &p, const PruneWork &w, int32_t nG, int32_t *rp,
                                  hipStream_t s) {
    if (p.vtype == ISING_I32) hipLaunchKernelGGL((k_csr_count<int32_t>), g1(nG), dim3(256), 0, s, p, w, nG, rp);
    else if (p.vtype == ISING_F32) hipLaunchKernelGGL((k_csr_count<float>), g1(nG), dim3(256), 0, s, p, w, nG, rp);
    else hipLaunchKernelGGL((k_csr_count<double>), g1(nG), dim3(256), 0, s, p, w, nG, rp);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, nG, rp, w.counts);
    return hipGetLastError();
}

hipError_t launch_prune_csr_fill(const DevProblem &p, const PruneWork &w, int32_t nG, const int32_t *rp,
                                 int32_t *colG, void *valG, void *hG, hipStream_t s) {
    if (p.vtype == ISING_I32)
        hipLaunchKernelGGL((k_csr_fill<int32_t, int64_t, int32_t>), g1(nG), dim3(256), 0, s, p, w, nG, rp, colG,
                           (int32_t *)valG, (int32_t *)hG);
    else if (p.vtype == ISING_F32)
        hipLaunchKernelGGL((k_csr_fill<float, double, double>), g1(nG), dim3(256), 0, s, p, w, nG, rp, colG,
                           (double *)valG, (double *)hG);
    else
        hipLaunchKernelGGL((k_csr_fill<double, double, double>), g1(nG), dim3(256), 0, s, p, w, nG, rp, colG,
                           (double *)valG, (double *)hG);
    return hipGetLastError();
}

hipError_t launch_unprune(const PruneWork &w, int32_t n, int32_t rounds, const int8_t *sG, int8_t *s_out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_unprune, dim3(1), dim3(1024), 0, s, w, n, rounds, sG, s_out);
    return hipGetLastError();
}

hipError_t launch_copy_record(const PruneWork &w, int32_t n, int8_t *kind, int32_t *round_of, int8_t *fixed,
                              int32_t *partner, int8_t *sigma, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_record, g1(n), dim3(256), 0, s, w, n, kind, round_of, fixed, partner, sigma);
    return hipGetLastError();
}

}  // namespace ising
