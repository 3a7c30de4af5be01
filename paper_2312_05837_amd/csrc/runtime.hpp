// Shared host runtime of the library: device buffer pools, contexts, pruning
// results, ingest, launch planning and the engines' host sides.  Used by the
// C ABI in api.cpp and by the serving loop in serve.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace ising {
namespace rt {

// Named device buffers that grow on demand and live until release().
struct Pool {
    struct Entry {
        void *p = nullptr;
        size_t bytes = 0;
    };
    std::map<std::string, Entry> m;
    size_t total = 0;
    hipError_t get(const std::string &key, size_t bytes, void **out) {
        Entry &e = m[key];
        if (bytes == 0) bytes = 8;
        if (e.bytes < bytes) {
            if (e.p) {
                hipError_t er = hipFree(e.p);
                if (er != hipSuccess) return er;
                total -= e.bytes;
            }
            e.p = nullptr;
            e.bytes = 0;
            hipError_t er = hipMalloc(&e.p, bytes);
            if (er != hipSuccess) return er;
            e.bytes = bytes;
            total += bytes;
        }
        *out = e.p;
        return hipSuccess;
    }
    void release() {
        for (auto &kv : m)
            if (kv.second.p) (void)hipFree(kv.second.p);
        m.clear();
        total = 0;
    }
    ~Pool() { release(); }
};

struct Server;

}  // namespace rt
}  // namespace ising

struct ising_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;           // written through set_error / read through error_copy only
    std::mutex err_mu;         // the scheduler thread of serving and waiting threads write it too
    std::string last_kernel;  // domain-selection kernel form of the last launch on this context
    ising::rt::Pool pool;
    std::mutex mu;
    ising::rt::Server *server = nullptr;
};

struct ising_pruned {
    int device = 0;
    int32_t n = 0, nG = 0, rounds = 0;
    int64_t nnzG = 0;
    int32_t vtype = ISING_I32;  // input value type
    int32_t format = ISING_DENSE;
    bool identity = true;
    double C = 0.0;
    ising::PruneWork w{};
    ising_problem reduced{};
    ising::rt::Pool own;        // buffers when the handle owns them
    ising::rt::Pool *pool = nullptr;
};

namespace ising {
namespace rt {

ising_status fail(ising_ctx *ctx, ising_status st, const std::string &msg);
// The context's last failure message, set and copied under its lock (ctx may be NULL).
void set_error(ising_ctx *ctx, const std::string &msg);
std::string error_copy(ising_ctx *ctx);

#define HIP_TRY(ctx, expr)                                                                     \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return ::ising::rt::fail((ctx), _e == hipErrorOutOfMemory ? ISING_ENOMEM : ISING_EDEVICE, \
                                     std::string(#expr) + ": " + hipGetErrorString(_e));       \
    } while (0)

#define ST_TRY(expr)                          \
    do {                                      \
        ising_status _s = (expr);             \
        if (_s != ISING_OK) return _s;        \
    } while (0)

ising_status check_problem_shape(ising_ctx *ctx, const ising_problem *p);
// Step size, weight of the L1 term and ADAM constants: lr and mu finite and > 0; for ADAM
// 0 <= beta1, beta2 < 1 and eps finite and > 0 (every bias correction and step denominator
// finite).  ctx may be NULL (no message).
ising_status check_params(ising_ctx *ctx, const ising_params &prm);
// Copy a host-buffer problem into device buffers of `pool` (keys prefixed by `prefix`) on
// stream s; *dev receives the same problem with device pointers.  Not synchronised.
ising_status upload_problem(ising_ctx *ctx, const ising_problem &host, Pool &pool, const std::string &prefix,
                            ising_problem &dev, hipStream_t s);

struct Ingest {
    int32_t flags[5] = {0, 0, 1, 1, 0};
    bool integer() const { return flags[3] != 0; }
    bool uniform_mag() const { return flags[2] != 0; }
    int maxdeg() const { return flags[1]; }
    int max_abs_int() const { return flags[4]; }  // largest |J| when J is integral
    double w = 1.0;
};

// Validate a device problem; fills the format facts (degree, common magnitude, integrality).
ising_status ingest(ising_ctx *ctx, const DevProblem &p, Pool &pool, Ingest &out, hipStream_t s);
// Algorithm 1 to completion on the device; pr.pool must be set.
ising_status prune_core(ising_ctx *ctx, const DevProblem &p, ising_pruned &pr, hipStream_t s);

struct DSPlan {
    DSLaunch l;
    bool packed = false;  // +-w couplings: sign-packed formats
    bool mult = false;    // small integer couplings: staged image with repeated entries, if it fits
};
// Launch plan of the persistent engine; with register_only the streaming form is never chosen.
ising_status plan_ds(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const Ingest &ing,
                     DSPlan &plan, bool register_only = false);
// Device formats and the problem/hyper-parameter fields of a DSArgs (state, steps left to the caller).
// batched: the plan is for the batched (serving) launches, which take at most 4 spins per thread.
ising_status prepare_ds(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const Ingest &ing,
                        Pool &pool, hipStream_t s, DSArgs &a, DSPlan &plan, bool register_only = false,
                        bool batched = false);
ising_status run_ds(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const Ingest &ing,
                    const void *uniform, int32_t t0, int32_t steps, ising_ds_state *st, Pool &pool,
                    hipStream_t s, hipEvent_t kbeg = nullptr, hipEvent_t kend = nullptr);
// Integer couplings that a one-byte matrix-core form holds exactly.  unit: w when all nonzero
// couplings are integers of one magnitude w and n w < 2^24 (every product of J / w with a vertex,
// and every partial sum, is then exact in FP8 x FP8 with FP32 accumulation), else 0.  imax: the
// largest |J| when the couplings are integers with |J| <= 127 and n |J| < 2^24 (one INT8 digit
// holds them; every sum is an integer below 2^24), else 0.
struct DenseExact {
    double unit = 0.0;
    int imax = 0;
};
DenseExact dense_exact(const Ingest &ing, int n);
// Operands of the matrix-core engine (split J) and the problem fields of a DenseRun.  An FP32
// request on exact integer couplings runs the FP8 form (one magnitude) or the INT8 form with
// one digit (several magnitudes up to 127): exact there, with the FP32 form's results.
ising_status prepare_dense(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, Pool &pool,
                           hipStream_t s, DenseRun &d, const DenseExact &ex);
ising_status run_dense(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const void *uniform,
                       int32_t t0, int32_t steps, ising_ds_state *st, Pool &pool, hipStream_t s,
                       const DenseExact &ex, hipEvent_t kbeg = nullptr, hipEvent_t kend = nullptr);
bool use_dense_engine(const ising_problem &p, const ising_params &prm);
double ms_between(hipEvent_t a, hipEvent_t b);

}  // namespace rt
}  // namespace ising
