// Host runtime behind include/ising.h: contexts, device buffers, ingest checks,
// the pruning round loop, the domain-selection launch and the whole-solve
// pipeline.  All arithmetic of the method runs in the kernels; this file only
// allocates, launches, synchronises and copies.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"

using namespace ising;
using namespace ising::rt;

namespace ising {
namespace rt {

void set_error(ising_ctx *ctx, const std::string &msg) {
    if (!ctx) return;
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    ctx->err = msg;
}

std::string error_copy(ising_ctx *ctx) {
    if (!ctx) return std::string();
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    return ctx->err;
}

ising_status fail(ising_ctx *ctx, ising_status st, const std::string &msg) {
    set_error(ctx, msg);
    return st;
}

ising_status check_problem_shape(ising_ctx *ctx, const ising_problem *p) {
    if (!p) return fail(ctx, ISING_EINVAL, "problem is NULL");
    if (p->n <= 0) return fail(ctx, ISING_EINVAL, "n must be positive");
    if (p->value_type < ISING_I32 || p->value_type > ISING_F64)
        return fail(ctx, ISING_EINVAL, "unknown value_type");
    if (p->format == ISING_DENSE) {
        if (!p->J) return fail(ctx, ISING_EINVAL, "dense problem without J");
    } else if (p->format == ISING_CSR) {
        if (!p->row_ptr || (p->nnz > 0 && (!p->col || !p->val)) || p->nnz < 0 || p->nnz > INT32_MAX)
            return fail(ctx, ISING_EINVAL, "malformed CSR pointers or nnz");
    } else {
        return fail(ctx, ISING_EINVAL, "unknown format");
    }
    return ISING_OK;
}

ising_status check_params(ising_ctx *ctx, const ising_params &prm) {
    if (!std::isfinite(prm.lr) || prm.lr <= 0) return fail(ctx, ISING_EINVAL, "lr must be finite and > 0");
    if (!std::isfinite(prm.mu) || prm.mu <= 0) return fail(ctx, ISING_EINVAL, "mu must be finite and > 0");
    if (prm.optimizer == ISING_OPT_ADAM && (!(prm.beta1 >= 0 && prm.beta1 < 1) || !(prm.beta2 >= 0 && prm.beta2 < 1) ||
                                            !std::isfinite(prm.eps) || prm.eps <= 0))
        return fail(ctx, ISING_EINVAL, "ADAM needs 0 <= beta1, beta2 < 1 and a finite eps > 0");
    return ISING_OK;
}

ising_status upload_problem(ising_ctx *ctx, const ising_problem &host, Pool &pool, const std::string &prefix,
                            ising_problem &d, hipStream_t s) {
    const int n = host.n;
    const size_t vs = vsize(host.value_type);
    d = host;
    void *buf = nullptr;
    if (host.format == ISING_DENSE) {
        HIP_TRY(ctx, pool.get(prefix + "J", (size_t)n * n * vs, &buf));
        HIP_TRY(ctx, hipMemcpyAsync(buf, host.J, (size_t)n * n * vs, hipMemcpyHostToDevice, s));
        d.J = buf;
    } else {
        void *rp = nullptr, *c = nullptr, *v = nullptr;
        HIP_TRY(ctx, pool.get(prefix + "rp", (size_t)(n + 1) * 4, &rp));
        HIP_TRY(ctx, pool.get(prefix + "col", (size_t)std::max<int64_t>(host.nnz, 1) * 4, &c));
        HIP_TRY(ctx, pool.get(prefix + "val", (size_t)std::max<int64_t>(host.nnz, 1) * vs, &v));
        HIP_TRY(ctx, hipMemcpyAsync(rp, host.row_ptr, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s));
        if (host.nnz > 0) {
            HIP_TRY(ctx, hipMemcpyAsync(c, host.col, (size_t)host.nnz * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(ctx, hipMemcpyAsync(v, host.val, (size_t)host.nnz * vs, hipMemcpyHostToDevice, s));
        }
        d.row_ptr = (const int32_t *)rp;
        d.col = (const int32_t *)c;
        d.val = v;
    }
    if (host.h) {
        void *hb = nullptr;
        HIP_TRY(ctx, pool.get(prefix + "h", (size_t)n * vs, &hb));
        HIP_TRY(ctx, hipMemcpyAsync(hb, host.h, (size_t)n * vs, hipMemcpyHostToDevice, s));
        d.h = hb;
    }
    return ISING_OK;
}

ising_status ingest(ising_ctx *ctx, const DevProblem &p, Pool &pool, Ingest &out, hipStream_t s) {
    void *flags = nullptr, *wdev = nullptr;
    HIP_TRY(ctx, pool.get("ingest.flags", 20, &flags));
    HIP_TRY(ctx, pool.get("ingest.w", 8, &wdev));
    HIP_TRY(ctx, launch_validate(p, (int32_t *)flags, (double *)wdev, s));
    HIP_TRY(ctx, hipMemcpyAsync(out.flags, flags, 20, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(&out.w, wdev, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const int bits = out.flags[0];
    if (bits & 1) return fail(ctx, ISING_EINVAL, "J is not symmetric");
    if (bits & 2) return fail(ctx, ISING_EINVAL, "J has a nonzero diagonal entry");
    if (bits & 4) return fail(ctx, ISING_EINVAL, "bad CSR structure (row_ptr, range or unsorted/duplicate columns)");
    if (bits & 8) return fail(ctx, ISING_EINVAL, "non-finite value in J or h");
    return ISING_OK;
}

// ---- pruning core ---------------------------------------------------------

ising_status prune_core(ising_ctx *ctx, const DevProblem &p, ising_pruned &pr, hipStream_t s) {
    Pool &pool = *pr.pool;
    const int n = p.n;
    const bool integer = p.vtype == ISING_I32;
    PruneWork &w = pr.w;
    auto g8 = [&](const char *k, int8_t **o) { return pool.get(std::string("pr.") + k, n, (void **)o); };
    auto g32 = [&](const char *k, int32_t **o) { return pool.get(std::string("pr.") + k, (size_t)n * 4, (void **)o); };
    HIP_TRY(ctx, g8("active", &w.active));
    HIP_TRY(ctx, g8("isD", &w.isD));
    HIP_TRY(ctx, g8("isS", &w.isS));
    HIP_TRY(ctx, g8("cand", &w.cand));
    HIP_TRY(ctx, g8("kind", &w.kind));
    HIP_TRY(ctx, g8("fixed", &w.fixed));
    HIP_TRY(ctx, g8("sigma", &w.sigma));
    HIP_TRY(ctx, g32("round", &w.round_of));
    HIP_TRY(ctx, g32("partner", &w.partner));
    HIP_TRY(ctx, g32("nb", &w.nb));
    HIP_TRY(ctx, g32("map", &w.map));
    HIP_TRY(ctx, g32("G", &w.G));
    HIP_TRY(ctx, pool.get("pr.h", (size_t)n * 8, &w.h));
    HIP_TRY(ctx, pool.get("pr.jv", (size_t)n * 8, &w.jv));
    HIP_TRY(ctx, pool.get("pr.cpart", (size_t)n * 8, &w.cpart));
    HIP_TRY(ctx, pool.get("pr.C", 8, &w.C));
    HIP_TRY(ctx, pool.get("pr.counts", 32, (void **)&w.counts));

    pr.n = n;
    pr.vtype = p.vtype;
    pr.format = p.format;
    HIP_TRY(ctx, launch_prune_init(p, w, s));
    // Rounds are enqueued in batches of 2, 4, 8, ... (at most 64): the round that removes
    // nothing raises a device-side flag that turns every later round into empty launches, so
    // the host reads the counters once per batch (once for most problems).  Every round
    // removes at least one spin, so at most n + 1 rounds run.
    int32_t counts[6] = {0, 0, 0, 0, 0, 0};
    int round = 0, batch = 2;
    for (;;) {
        for (int b = 0; b < batch; ++b) HIP_TRY(ctx, launch_prune_round(p, w, round++, s));
        HIP_TRY(ctx, hipMemcpyAsync(counts, w.counts, 24, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        if (counts[4]) break;
        if (round > n + 1) return fail(ctx, ISING_EDEVICE, "pruning did not terminate");
        batch = std::min(2 * batch, 64);
    }
    pr.rounds = counts[5];
    if (integer) {
        int64_t c = 0;
        HIP_TRY(ctx, hipMemcpyAsync(&c, w.C, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        pr.C = (double)c;
    } else {
        HIP_TRY(ctx, hipMemcpyAsync(&pr.C, w.C, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    HIP_TRY(ctx, launch_prune_compact_scan(p, w, s));
    HIP_TRY(ctx, hipMemcpyAsync(counts, w.counts, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const int nG = counts[2];
    pr.nG = nG;
    pr.identity = (nG == n);
    ising_problem &r = pr.reduced;
    std::memset(&r, 0, sizeof(r));
    if (pr.identity) {
        r.n = n;
        r.format = p.format;
        r.value_type = p.vtype;
        r.nnz = p.nnz;
        r.J = p.J;
        r.row_ptr = p.row_ptr;
        r.col = p.col;
        r.val = p.val;
        r.h = p.h;
        pr.nnzG = p.format == ISING_CSR ? p.nnz : 0;
        return ISING_OK;
    }
    const int ovt = integer ? ISING_I32 : ISING_F64;
    const size_t osz = integer ? 4 : 8;
    r.n = nG;
    r.format = p.format;
    r.value_type = ovt;
    if (nG == 0) {
        pr.nnzG = 0;
        return ISING_OK;
    }
    void *hG = nullptr;
    HIP_TRY(ctx, pool.get("pr.hG", (size_t)nG * osz, &hG));
    r.h = hG;
    if (p.format == ISING_DENSE) {
        void *JG = nullptr;
        HIP_TRY(ctx, pool.get("pr.JG", (size_t)nG * nG * osz, &JG));
        HIP_TRY(ctx, launch_prune_gather_dense(p, w, nG, JG, hG, s));
        r.J = JG;
        pr.nnzG = 0;
    } else {
        int32_t *rp = nullptr;
        HIP_TRY(ctx, pool.get("pr.rpG", (size_t)(nG + 1) * 4, (void **)&rp));
        HIP_TRY(ctx, launch_prune_csr_count(p, w, nG, rp, s));
        HIP_TRY(ctx, hipMemcpyAsync(counts, w.counts, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        const int64_t nnzG = counts[3];
        int32_t *cG = nullptr;
        void *vG = nullptr;
        HIP_TRY(ctx, pool.get("pr.colG", (size_t)std::max<int64_t>(nnzG, 1) * 4, (void **)&cG));
        HIP_TRY(ctx, pool.get("pr.valG", (size_t)std::max<int64_t>(nnzG, 1) * osz, &vG));
        HIP_TRY(ctx, launch_prune_csr_fill(p, w, nG, rp, cG, vG, hG, s));
        r.row_ptr = rp;
        r.col = cG;
        r.val = vG;
        r.nnz = nnzG;
        pr.nnzG = nnzG;
    }
    return ISING_OK;
}

// ---- domain-selection launch planning -------------------------------------

ising_status plan_ds(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const Ingest &ing,
                     DSPlan &plan, bool register_only) {
    ST_TRY(check_params(ctx, prm));
    const bool fp64 = prm.precision == ISING_PREC_FP64;
    if (prm.precision != ISING_PREC_FP64 && prm.precision != ISING_PREC_FP32)
        return fail(ctx, ISING_ENOTSUP, "precision not supported by the persistent engine");
    const int n = p.n, R = prm.replicas;
    if (n > ds_max_n(fp64)) return fail(ctx, ISING_ENOTSUP, "n exceeds the on-chip vertex-buffer limit");
    if (prm.loss != ISING_LOSS_VERTEX && prm.loss != ISING_LOSS_RELAXED) return fail(ctx, ISING_EINVAL, "unknown loss");
    const bool relaxed = prm.loss == ISING_LOSS_RELAXED;
    if (relaxed) register_only = true;  // sin(theta) is kept in LDS next to the vertex
    const bool conv = prm.conv_tol > 0;
    if (conv && (prm.conv_window < 1 || prm.conv_window > kConvWindowMax))
        return fail(ctx, ISING_EINVAL, "conv_window must be in 1..8");
    if (conv) register_only = true;  // the test runs in the register-resident engine
    DSLaunch &l = plan.l;
    l.fp64 = fp64;
    l.relaxed = relaxed;
    l.conv = conv;
    plan.packed = p.format == ISING_CSR && ing.uniform_mag();
    // small integer couplings (|J| <= kPmsMaxMult, not all equal) can still be staged, each
    // coupling repeated |J| times with unit magnitude; they keep CSR values if the image does not fit
    plan.mult = p.format == ISING_CSR && !plan.packed && ing.integer() && ing.max_abs_int() >= 1 &&
                ing.max_abs_int() <= kPmsMaxMult;
    l.coupling = p.format == ISING_DENSE ? CK_DENSE : (plan.packed ? CK_PM : CK_CSRV);
    // register-resident engine while at most 4 (spin, replica) elements per thread
    // fit, else the streaming engine; replicas per workgroup chosen so that there
    // are at least as many workgroups as compute units where R allows it
    int rg = 1;
    if (!fp64) {
        for (int cand : {4, 2}) {
            if (R % cand) continue;
            if (R / cand < 256) continue;
            if (plan.packed && cand == 4 && ing.maxdeg() > 255) continue;
            if (plan.mult && cand == 4 && (int64_t)ing.maxdeg() * ing.max_abs_int() > 255) plan.mult = false;
            rg = cand;
            break;
        }
    }
    // register-resident engine: up to 4 spins per thread (2 with four replicas per workgroup);
    // sparse FP32 problems with one replica per workgroup take up to 32 spins per thread, which
    // keeps a whole replica of n = 24576 spins in one CU's registers
    const bool wide = !fp64 && p.format == ISING_CSR;
    int ept = 0;
    for (;;) {
        const int maxept = fp64 ? 2 : (rg == 4 ? 2 : (rg == 2 || !wide ? 4 : 32));
        for (int e : {1, 2, 4, 8, 16, 28, 32}) {
            if (e > maxept) break;
            if ((int64_t)e * ds_block_limit(e) >= n) {
                ept = e;
                break;
            }
        }
        if (ept || rg == 1 || (!register_only && !wide)) break;
        rg = rg == 4 ? 2 : 1;  // fewer replicas per workgroup leave room for more spins per thread
    }
    if (ept == 0 && register_only)
        return fail(ctx, ISING_ENOTSUP,
                    relaxed ? "the relaxed loss needs the register-resident engine (n too large)"
                            : "n too large for the register-resident engine");
    if (ept == 0) {
        // streaming: spins triple-buffered in LDS
        const size_t sw = rg == 1 ? 1 : 4;
        while (rg > 1 && (size_t)3 * n * sw > 120 * 1024) {
            rg /= 2;
            if (R % rg) rg = 1;
        }
        if ((size_t)3 * n * (rg == 1 ? 1 : 4) > 150 * 1024)
            return fail(ctx, ISING_ENOTSUP, "n too large for the on-chip vertex buffers");
        l.rg = rg;
        l.ept = 0;
        l.block = 1024;
        return ISING_OK;
    }
    l.rg = rg;
    l.ept = ept;
    const int per = (n + ept - 1) / ept;
    l.block = std::max(64, (per + 63) / 64 * 64);
    return ISING_OK;
}

ising_status prepare_ds(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const Ingest &ing,
                        Pool &pool, hipStream_t s, DSArgs &a, DSPlan &plan, bool register_only, bool batched) {
    if (prm.replicas <= 0) return fail(ctx, ISING_EINVAL, "bad replicas");
    if (prm.optimizer != ISING_OPT_GD && prm.optimizer != ISING_OPT_ADAM)
        return fail(ctx, ISING_EINVAL, "unknown optimizer");
    ST_TRY(plan_ds(ctx, p, prm, ing, plan, register_only));
    const bool fp64 = plan.l.fp64;
    const size_t real = fp64 ? 8 : 4;
    const DevProblem dp = to_dev(p);
    a = DSArgs();
    a.n = p.n;
    a.R = prm.replicas;
    a.opt = prm.optimizer;
    a.seed = prm.seed;
    a.lr = prm.lr;
    a.mu = prm.mu;
    a.b1 = prm.beta1;
    a.b2 = prm.beta2;
    a.eps = prm.eps;
    a.w = ing.w;
    const int64_t total = p.format == ISING_DENSE ? (int64_t)p.n * p.n : p.nnz;
    void *fmt = nullptr, *hbuf = nullptr;
    HIP_TRY(ctx, pool.get("ds.fmt", (size_t)std::max<int64_t>(total, 1) * (plan.packed ? 4 : real), &fmt));
    if (p.h) HIP_TRY(ctx, pool.get("ds.h", (size_t)p.n * real, &hbuf));
    HIP_TRY(ctx, launch_ds_format(dp, fp64, plan.packed, (uint32_t *)fmt, fmt, p.h ? hbuf : nullptr, s));
    a.row_ptr = p.row_ptr;
    a.col = p.col;
    a.loss = prm.loss;
    a.conv_tol = prm.conv_tol > 0 ? prm.conv_tol : 0.0;
    a.conv_window = prm.conv_window;
    // Small problems with +-w couplings of degree <= 4 (tori, 3-regular graphs): the fixed-width-row
    // form with one replica per workgroup of four wavefronts and 4 or 8 spins per thread, instead
    // of the staged image (which puts four replicas in a workgroup and gathers through LDS)
    bool small_rows = false;
    if (plan.packed && !batched && !fp64 && !plan.l.relaxed && ing.maxdeg() <= kEllWidth && pme_small_ept(p.n) > 0 &&
        plan.l.ept > 0) {
        small_rows = true;
        plan.l.coupling = CK_PM;
        plan.l.rg = 1;
        plan.l.ept = pme_small_ept(p.n);
        plan.l.block = kPmeSmallBlock;
    }
    if (!small_rows && (plan.packed || plan.mult) && plan.l.ept > 0 && plan.l.ept <= 8) {
        const double wunit = plan.packed ? ing.w : 1.0;
        // stage the +-w couplings in LDS when the image fits next to the vertex buffers (and,
        // for the relaxed loss, next to sin(theta) and its negation)
        DSLaunch l2 = plan.l;
        l2.coupling = CK_PMS;
        const int rb = pms_region_bytes(l2);
        const int slots = l2.ept * l2.block;
        if (2 * (int64_t)rb <= 65536 && slots / 64 <= 256) {
            PmsWork w;
            HIP_TRY(ctx, pool.get("ds.pms.deg", (size_t)p.n * 4, (void **)&w.deg));
            HIP_TRY(ctx, pool.get("ds.pms.pos", (size_t)p.n * 4, (void **)&w.pos));
            HIP_TRY(ctx, pool.get("ds.pms.perm", (size_t)slots * 4, (void **)&w.perm));
            HIP_TRY(ctx, pool.get("ds.pms.prow", (size_t)slots * 4, (void **)&w.prow));
            HIP_TRY(ctx, pool.get("ds.pms.pcnt", (size_t)slots * 4, (void **)&w.pcnt));
            HIP_TRY(ctx, pool.get("ds.pms.total", 4, (void **)&w.total));
            int32_t total = 0;
            HIP_TRY(ctx, launch_pms_format(dp, l2, wunit, w, &total, s));
            if (ds_lds_bytes(l2, p.n, total) <= 160 * 1024) {
                HIP_TRY(ctx, pool.get("ds.pms.img", (size_t)std::max(total, 1) * 8, (void **)&w.img));
                HIP_TRY(ctx, launch_pms_format(dp, l2, wunit, w, &total, s));
                plan.l = l2;
                a.pimg = w.img;
                a.pimg_groups = total;
                a.prow = w.prow;
                a.pcnt = w.pcnt;
                a.pperm = w.perm;
                a.pms_rb = rb;
                a.w = wunit;
            }
        }
    }
    if (plan.packed) a.pm = (const uint32_t *)fmt;
    // wide packed engine (one replica per workgroup, 8+ spins per thread): fixed-width neighbour
    // rows and a per-position field, loaded ahead of each spin's update, when every degree fits
    // them; the workgroup is then the launch bound of its spins per thread
    if (plan.packed && plan.l.coupling == CK_PM && (plan.l.ept >= 8 || small_rows) && plan.l.rg == 1 && !plan.l.relaxed &&
        ing.maxdeg() <= kEllWidth && (int64_t)plan.l.ept * ds_block_limit(plan.l.ept) < 32768) {
        if (!small_rows) plan.l.block = ds_block_limit(plan.l.ept);
        void *ell = nullptr, *hrow = nullptr;
        const size_t pos = (size_t)plan.l.ept * plan.l.block;
        HIP_TRY(ctx, pool.get("ds.ell", pos * kEllWidth * 4, &ell));
        HIP_TRY(ctx, pool.get("ds.ell.h", pos * 4, &hrow));
        HIP_TRY(ctx, launch_ell_format(dp, (const uint32_t *)fmt, p.h ? (const float *)hbuf : nullptr, plan.l.ept,
                                       plan.l.block, (uint32_t *)ell, (float *)hrow, s));
        a.ell = (const uint32_t *)ell;
        a.ellh = (const float *)hrow;
    }
    else if (p.format == ISING_CSR) a.val = fmt;
    else a.J = fmt;
    a.h = p.h ? hbuf : nullptr;
    {
        // no field and integer couplings whose |J| summed over all entries stays below 2^24:
        // every product and energy sum of the FP32 engine is then an exact integer
        const double jmax = ing.uniform_mag() ? ing.w : (double)ing.max_abs_int();
        const double entries = p.format == ISING_CSR ? (double)p.nnz : (double)p.n * p.n;
        a.exact_sums = !p.h && ing.integer() && jmax > 0 && jmax * entries < 16777216.0;
    }
    return ISING_OK;
}

ising_status run_ds(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const Ingest &ing,
                    const void *uniform, int32_t t0, int32_t steps, ising_ds_state *st, Pool &pool,
                    hipStream_t s, hipEvent_t kbeg, hipEvent_t kend) {
    if (steps < 0 || t0 < 0) return fail(ctx, ISING_EINVAL, "bad steps/t0");
    if (!st || !st->theta || !st->s_best || !st->e_best || !st->best_step)
        return fail(ctx, ISING_EINVAL, "state buffers missing");
    if (prm.optimizer == ISING_OPT_ADAM && (!st->m || !st->v))
        return fail(ctx, ISING_EINVAL, "ADAM needs m and v buffers");
    if (prm.conv_tol > 0 && t0 != 0 && (!st->conv_step || !st->conv_state))
        return fail(ctx, ISING_EINVAL, "continuing the convergence test (t0 > 0) needs conv_step and conv_state");
    DSArgs a;
    DSPlan plan;
    ST_TRY(prepare_ds(ctx, p, prm, ing, pool, s, a, plan));
    const bool fp64 = plan.l.fp64;
    const size_t real = fp64 ? 8 : 4;
    a.t0 = t0;
    a.steps = steps;
    a.init_mode = t0 > 0 ? 0 : (uniform ? 1 : 2);
    a.theta = st->theta;
    a.m = prm.optimizer == ISING_OPT_ADAM ? st->m : nullptr;
    a.v = prm.optimizer == ISING_OPT_ADAM ? st->v : nullptr;
    a.uniform = uniform;
    a.s_best = st->s_best;
    a.e_best = st->e_best;
    a.best_step = st->best_step;
    a.etrace = st->energy_trace;
    a.ltrace = st->loss_trace;
    a.conv_step = st->conv_step;
    a.conv_state = st->conv_state;
    if (prm.optimizer == ISING_OPT_ADAM && steps > 0) {
        void *bias = nullptr;
        HIP_TRY(ctx, pool.get("ds.bias", (size_t)2 * steps * real, &bias));
        HIP_TRY(ctx, launch_bias_table(prm.beta1, prm.beta2, t0, steps, fp64, bias, s));
        a.bias = bias;
    }
    if (kbeg) HIP_TRY(ctx, hipEventRecord(kbeg, s));
    hipError_t e = launch_ds(a, plan.l, s, &ctx->last_kernel);
    if (kend && e == hipSuccess) HIP_TRY(ctx, hipEventRecord(kend, s));
    if (e != hipSuccess)
        return fail(ctx, e == hipErrorInvalidValue ? ISING_ENOTSUP : ISING_EDEVICE,
                    std::string("domain-selection launch: ") + hipGetErrorString(e));
    return ISING_OK;
}

constexpr int kDenseInt8MaxN = 65536;

ising_status prepare_dense(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, Pool &pool,
                           hipStream_t s, DenseRun &d, const DenseExact &ex) {
    const double unit = ex.unit;
    ST_TRY(check_params(ctx, prm));
    if (p.format != ISING_DENSE) return fail(ctx, ISING_ENOTSUP, "the matrix-core engine needs dense couplings");
    if (prm.loss != ISING_LOSS_VERTEX) return fail(ctx, ISING_ENOTSUP, "the matrix-core engine runs the vertex loss");
    if (prm.conv_tol > 0) return fail(ctx, ISING_ENOTSUP, "the matrix-core engine runs fixed step counts");
    int form;
    // couplings of one integer magnitude w: J / w and the vertex are exact in FP8 and every
    // product and partial sum is an integer below 2^24, so the FP8 form gives the FP32
    // form's results bit for bit
    // couplings that are integers up to 127 of several magnitudes: one INT8 digit holds them and
    // every sum is an integer below 2^24, so that form gives the FP32 form's results too
    if (prm.precision == ISING_PREC_FP32 && unit > 0) form = DF_FP8;
    else if (prm.precision == ISING_PREC_FP32 && ex.imax > 0) form = DF_I8X1;
    else if (prm.precision == ISING_PREC_FP32) form = DF_FP32;
    else if (prm.precision == ISING_PREC_BF16X2) form = DF_BF16X2;
    else if (prm.precision == ISING_PREC_BF16) form = DF_BF16;
    else if (prm.precision == ISING_PREC_FP8 && unit > 0) form = DF_FP8;
    else if (prm.precision == ISING_PREC_FP8)
        return fail(ctx, ISING_ENOTSUP, "the FP8 form needs couplings of one integer magnitude w with n w < 2^24");
    else if (prm.precision == ISING_PREC_I8X3) form = DF_I8X3;
    else if (prm.precision == ISING_PREC_I8X2) form = DF_I8X2;
    else return fail(ctx, ISING_ENOTSUP, "the matrix-core engine runs FP32, BF16X2, BF16, FP8, I8X3 or I8X2");
    // INT8 forms: every partial sum stays below 2^31 only while 257 n is well below it
    if ((form == DF_I8X3 || form == DF_I8X2 || form == DF_I8X1) && p.n > kDenseInt8MaxN)
        return fail(ctx, ISING_ENOTSUP, "the INT8 forms take n <= 65536");
    if (prm.replicas <= 0) return fail(ctx, ISING_EINVAL, "bad replicas");
    if (prm.optimizer != ISING_OPT_GD && prm.optimizer != ISING_OPT_ADAM)
        return fail(ctx, ISING_EINVAL, "unknown optimizer");
    const int n = p.n, R = prm.replicas;
    d = DenseRun();
    d.n = n;
    d.R = R;
    d.Mp = (n + 127) / 128 * 128;
    // the K loops read 128 bytes of each row per chunk: 64 BF16 or 128 FP8 / INT8 values
    const bool bytes = form == DF_FP8 || form == DF_I8X3 || form == DF_I8X2 || form == DF_I8X1;
    d.Kp = bytes ? (n + 127) / 128 * 128 : (n + 63) / 64 * 64;
    d.jscale = form == DF_FP8 ? (float)unit : 1.f;
    d.form = form;
    d.opt = prm.optimizer;
    d.seed = prm.seed;
    d.lr = prm.lr;
    d.mu = prm.mu;
    d.b1 = prm.beta1;
    d.b2 = prm.beta2;
    d.eps = prm.eps;
    void *Jhi = nullptr, *Jlo = nullptr, *Jf = nullptr, *hf = nullptr, *S = nullptr, *Ep = nullptr, *Lp = nullptr;
    void *jsc = nullptr;
    const size_t mk = (size_t)d.Mp * d.Kp;
    if (form == DF_FP32) {
        HIP_TRY(ctx, pool.get("dn.Jf", mk * 4, &Jf));
    } else if (form == DF_BF16X2) {
        HIP_TRY(ctx, pool.get("dn.Jhi", mk * 2, &Jhi));
        HIP_TRY(ctx, pool.get("dn.Jlo", mk * 2, &Jlo));
    } else {
        HIP_TRY(ctx, pool.get("dn.Jhi", mk * dense_j_bytes(form), &Jhi));  // (INT8: the digit planes)
    }
    if (form == DF_I8X3 || form == DF_I8X2 || form == DF_I8X1) HIP_TRY(ctx, pool.get("dn.jsc", kDenseScaleBytes, &jsc));
    if (p.h) HIP_TRY(ctx, pool.get("dn.h", (size_t)n * 4, &hf));
    HIP_TRY(ctx, pool.get("dn.S", (size_t)kDenseVertexBufs * R * d.Kp * dense_vertex_bytes(form), &S));
    HIP_TRY(ctx, pool.get("dn.Ep", (size_t)2 * (d.Mp / 128) * R * 4, &Ep));
    HIP_TRY(ctx, pool.get("dn.Lp", (size_t)2 * (d.Mp / 128) * R * 4, &Lp));
    HIP_TRY(ctx, launch_dense_prepare(to_dev(p), form, d.Mp, d.Kp, Jhi, Jlo, Jf, (float *)hf, jsc, s));
    d.jsc = jsc;
    d.Jhi = Jhi;
    d.Jlo = Jlo;
    d.Jf = Jf;
    d.h = p.h ? (const float *)hf : nullptr;
    d.S = S;
    d.Epart = (float *)Ep;
    d.Lpart = (float *)Lp;
    return ISING_OK;
}

ising_status run_dense(ising_ctx *ctx, const ising_problem &p, const ising_params &prm, const void *uniform,
                       int32_t t0, int32_t steps, ising_ds_state *st, Pool &pool, hipStream_t s,
                       const DenseExact &ex, hipEvent_t kbeg, hipEvent_t kend) {
    if (steps < 0 || t0 < 0) return fail(ctx, ISING_EINVAL, "bad steps/t0");
    if (!st || !st->theta || !st->s_best || !st->e_best || !st->best_step)
        return fail(ctx, ISING_EINVAL, "state buffers missing");
    if (prm.optimizer == ISING_OPT_ADAM && (!st->m || !st->v)) return fail(ctx, ISING_EINVAL, "ADAM needs m and v");
    DenseRun d;
    ST_TRY(prepare_dense(ctx, p, prm, pool, s, d, ex));
    d.t0 = t0;
    d.steps = steps;
    d.init_mode = t0 > 0 ? 0 : (uniform ? 1 : 2);
    d.uniform = uniform;
    if (prm.optimizer == ISING_OPT_ADAM && steps > 0) {
        void *bias = nullptr;
        HIP_TRY(ctx, pool.get("dn.bias", (size_t)2 * steps * 4, &bias));
        HIP_TRY(ctx, launch_bias_table(prm.beta1, prm.beta2, t0, steps, false, bias, s));
        d.bias = (const float *)bias;
    }
    d.theta = (float *)st->theta;
    d.m = prm.optimizer == ISING_OPT_ADAM ? (float *)st->m : nullptr;
    d.v = prm.optimizer == ISING_OPT_ADAM ? (float *)st->v : nullptr;
    d.e_best = st->e_best;
    d.best_step = st->best_step;
    d.s_best = st->s_best;
    d.etrace = st->energy_trace;
    d.ltrace = st->loss_trace;
    void *scratch = nullptr;
    const DenseRun *one = &d;
    HIP_TRY(ctx, pool.get("dn.group", dense_group_scratch_bytes(&one, 1), &scratch));
    if (kbeg) HIP_TRY(ctx, hipEventRecord(kbeg, s));
    hipError_t e = launch_dense_run(d, scratch, s);
    static const char *const forms[] = {"fp32", "bf16x2", "bf16", "fp8", "i8x3", "i8x2", "i8x1"};
    ctx->last_kernel = std::string("k_dense_step<") + forms[d.form] + ">";
    if (e != hipSuccess)
        return fail(ctx, e == hipErrorInvalidValue ? ISING_ENOTSUP : ISING_EDEVICE,
                    std::string("matrix-core domain selection: ") + hipGetErrorString(e));
    if (kend) HIP_TRY(ctx, hipEventRecord(kend, s));
    return ISING_OK;
}

// dense problems with more than this many spins use the matrix-core engine in FP32
constexpr int kDenseMfmaMinN = 256;  // n above which dense FP32 problems use MFMA

bool use_dense_engine(const ising_problem &p, const ising_params &prm) {
    if (p.format != ISING_DENSE || prm.loss != ISING_LOSS_VERTEX || prm.conv_tol > 0) return false;
    if (prm.precision == ISING_PREC_BF16X2 || prm.precision == ISING_PREC_BF16 || prm.precision == ISING_PREC_FP8 ||
        prm.precision == ISING_PREC_I8X3 || prm.precision == ISING_PREC_I8X2)
        return true;
    return prm.precision == ISING_PREC_FP32 && p.n > kDenseMfmaMinN;
}

DenseExact dense_exact(const Ingest &ing, int n) {
    DenseExact ex;
    ex.unit = ing.integer() && ing.uniform_mag() && (double)n * ing.w < 16777216.0 ? ing.w : 0.0;
    const int m = ing.integer() ? ing.max_abs_int() : 0;
    ex.imax = m >= 1 && m <= 127 && (double)n * m < 16777216.0 ? m : 0;
    return ex;
}

double ms_between(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms;
}

}  // namespace rt
}  // namespace ising

extern "C" {

ising_status ising_create(int device, ising_ctx **out) {
    if (!out) return ISING_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ISING_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return ISING_EDEVICE;
    auto *c = new (std::nothrow) ising_ctx();
    if (!c) return ISING_ENOMEM;
    c->device = device;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return ISING_EDEVICE;
    }
    // the static scratch of ising_energy_dev_noalloc: its address on this device, once
    void *scratch = nullptr;
    if (energy_scratch_address(device, &scratch) != hipSuccess) {
        (void)hipStreamDestroy(c->stream);
        delete c;
        return ISING_EDEVICE;
    }
    *out = c;
    return ISING_OK;
}

ising_status ising_destroy(ising_ctx *ctx) {
    if (!ctx) return ISING_OK;
    if (ctx->server) (void)ising_serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipDeviceSynchronize();
    ctx->pool.release();
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return ISING_OK;
}

const char *ising_last_error(const ising_ctx *ctx) {
    // a copy per calling thread, valid until that thread's next call of this function
    thread_local std::string copy;
    if (!ctx) return "no context";
    copy = error_copy(const_cast<ising_ctx *>(ctx));
    return copy.c_str();
}

const char *ising_last_kernel(const ising_ctx *ctx) { return ctx ? ctx->last_kernel.c_str() : ""; }

ising_status ising_energy(ising_ctx *ctx, const ising_problem *problem, const int8_t *spins, int32_t count,
                          double *E_out, int64_t *E_int_out) {
    if (!ctx) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    if (count < 0 || (count > 0 && !spins)) return fail(ctx, ISING_EINVAL, "bad spins/count");
    if (E_int_out && problem->value_type != ISING_I32)
        return fail(ctx, ISING_EINVAL, "integer energies need an ISING_I32 problem");
    if (count == 0) return ISING_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    Pool &pool = ctx->pool;
    ising_problem d;
    ST_TRY(upload_problem(ctx, *problem, pool, "en.", d, s));
    const size_t sb = (size_t)count * problem->n;
    void *sdev = nullptr, *edev = nullptr, *eidev = nullptr, *partial = nullptr;
    HIP_TRY(ctx, pool.get("en.s", sb, &sdev));
    HIP_TRY(ctx, pool.get("en.E", (size_t)count * 8, &edev));
    HIP_TRY(ctx, pool.get("en.Ei", (size_t)count * 8, &eidev));
    HIP_TRY(ctx, pool.get("energy.partial", energy_partial_bytes(problem->n, count), &partial));
    HIP_TRY(ctx, hipMemcpyAsync(sdev, spins, sb, hipMemcpyHostToDevice, s));
    const bool want_int = problem->value_type == ISING_I32;
    HIP_TRY(ctx, launch_energy(to_dev(d), (const int8_t *)sdev, count, partial, (double *)edev,
                               want_int ? (int64_t *)eidev : nullptr, s));
    if (E_out) HIP_TRY(ctx, hipMemcpyAsync(E_out, edev, (size_t)count * 8, hipMemcpyDeviceToHost, s));
    if (E_int_out) HIP_TRY(ctx, hipMemcpyAsync(E_int_out, eidev, (size_t)count * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return ISING_OK;
}

ising_status ising_energy_dev_noalloc(ising_ctx *ctx, const ising_problem *problem, const int8_t *spins,
                                      int32_t count, double *E_out, int64_t *E_int_out, void *stream) {
    if (!ctx) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    if (count < 0 || (count > 0 && !spins)) return fail(ctx, ISING_EINVAL, "bad spins/count");
    if (E_int_out && problem->value_type != ISING_I32)
        return fail(ctx, ISING_EINVAL, "integer energies need an ISING_I32 problem");
    if (energy_partial_bytes(problem->n, count) > kEnergyScratchBytes)
        return fail(ctx, ISING_EINVAL,
                    "count * ceil(n / 4) * 8 bytes of partial sums exceed the static scratch of " +
                        std::to_string(kEnergyScratchBytes) + " bytes");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    void *partial = nullptr;
    HIP_TRY(ctx, energy_scratch_address(ctx->device, &partial));
    HIP_TRY(ctx, launch_energy(to_dev(*problem), spins, count, partial, E_out, E_int_out, (hipStream_t)stream));
    return ISING_OK;
}

ising_status ising_prune(ising_ctx *ctx, const ising_problem *problem, ising_pruned **out) {
    if (!ctx || !out) return ISING_EINVAL;
    *out = nullptr;
    ST_TRY(check_problem_shape(ctx, problem));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    auto pr = std::make_unique<ising_pruned>();
    pr->device = ctx->device;
    pr->pool = &pr->own;
    ising_problem d;  // the handle owns this device copy (its reduced problem may alias it)
    ST_TRY(upload_problem(ctx, *problem, pr->own, "in.", d, s));
    Ingest ing;
    ST_TRY(ingest(ctx, to_dev(d), ctx->pool, ing, s));
    ST_TRY(prune_core(ctx, to_dev(d), *pr, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *out = pr.release();
    return ISING_OK;
}

ising_status ising_unprune(const ising_pruned *pr, const int8_t *s_G, int8_t *s_out) {
    if (!pr || !s_out || (pr->nG > 0 && !s_G)) return ISING_EINVAL;
    if (hipSetDevice(pr->device) != hipSuccess) return ISING_EDEVICE;
    const size_t n = (size_t)pr->n, nG = (size_t)pr->nG;
    int8_t *buf = nullptr;
    if (hipMalloc((void **)&buf, n + std::max<size_t>(nG, 1)) != hipSuccess) return ISING_ENOMEM;
    int8_t *dsG = buf + n;
    hipError_t e = nG ? hipMemcpy(dsG, s_G, nG, hipMemcpyHostToDevice) : hipSuccess;
    if (e == hipSuccess)
        e = pr->identity ? hipMemcpy(buf, dsG, n, hipMemcpyDeviceToDevice)
                         : launch_unprune(pr->w, pr->n, pr->rounds, dsG, buf, nullptr);
    if (e == hipSuccess) e = hipMemcpy(s_out, buf, n, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    return e == hipSuccess ? ISING_OK : ISING_EDEVICE;
}

ising_status ising_pruned_record(const ising_pruned *pr, int8_t *kind, int32_t *round_of, int8_t *fixed,
                                 int32_t *partner, int8_t *sigma, int32_t *G, void *h_G) {
    if (!pr) return ISING_EINVAL;
    if (hipSetDevice(pr->device) != hipSuccess) return ISING_EDEVICE;
    const size_t n = (size_t)pr->n;
    void *buf = nullptr;
    if (hipMalloc(&buf, n * 11 + 4) != hipSuccess) return ISING_ENOMEM;
    int8_t *dk = (int8_t *)buf, *df = dk + n, *ds = df + n;
    int32_t *dr = (int32_t *)(ds + n + (4 - (3 * n) % 4) % 4), *dp = dr + n;
    hipError_t e = launch_copy_record(pr->w, pr->n, dk, dr, df, dp, ds, nullptr);
    if (e == hipSuccess && kind) e = hipMemcpy(kind, dk, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && round_of) e = hipMemcpy(round_of, dr, n * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && fixed) e = hipMemcpy(fixed, df, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && partner) e = hipMemcpy(partner, dp, n * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sigma) e = hipMemcpy(sigma, ds, n, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (e != hipSuccess) return ISING_EDEVICE;
    if (G && pr->nG > 0) {
        if (pr->identity) {
            for (int32_t i = 0; i < pr->n; ++i) G[i] = i;
        } else if (hipMemcpy(G, pr->w.G, (size_t)pr->nG * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            return ISING_EDEVICE;
        }
    }
    if (h_G && pr->nG > 0 && pr->reduced.h &&
        hipMemcpy(h_G, pr->reduced.h, (size_t)pr->nG * vsize(pr->reduced.value_type), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return ISING_EDEVICE;
    return ISING_OK;
}

ising_status ising_pruned_copy(const ising_pruned *pr, void *J_or_val, int32_t *row_ptr, int32_t *col, void *h) {
    if (!pr) return ISING_EINVAL;
    if (hipSetDevice(pr->device) != hipSuccess) return ISING_EDEVICE;
    const ising_problem &r = pr->reduced;
    if (r.n == 0) return ISING_OK;
    const size_t vs = vsize(r.value_type);
    hipError_t e = hipSuccess;
    if (r.format == ISING_DENSE) {
        if (J_or_val) e = hipMemcpy(J_or_val, r.J, (size_t)r.n * r.n * vs, hipMemcpyDeviceToHost);
    } else {
        if (row_ptr) e = hipMemcpy(row_ptr, r.row_ptr, (size_t)(r.n + 1) * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && col && r.nnz) e = hipMemcpy(col, r.col, (size_t)r.nnz * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && J_or_val && r.nnz)
            e = hipMemcpy(J_or_val, r.val, (size_t)r.nnz * vs, hipMemcpyDeviceToHost);
    }
    if (e == hipSuccess && h && r.h) e = hipMemcpy(h, r.h, (size_t)r.n * vs, hipMemcpyDeviceToHost);
    return e == hipSuccess ? ISING_OK : ISING_EDEVICE;
}

ising_status ising_energy_dev(ising_ctx *ctx, const ising_problem *problem, const int8_t *spins, int32_t count,
                              double *E_out, int64_t *E_int_out, void *stream) {
    if (!ctx) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    if (count < 0 || (count > 0 && !spins)) return fail(ctx, ISING_EINVAL, "bad spins/count");
    if (E_int_out && problem->value_type != ISING_I32)
        return fail(ctx, ISING_EINVAL, "integer energies need an ISING_I32 problem");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    void *partial = nullptr;
    HIP_TRY(ctx, ctx->pool.get("energy.partial", energy_partial_bytes(problem->n, count), &partial));
    HIP_TRY(ctx, launch_energy(to_dev(*problem), spins, count, partial, E_out, E_int_out, s));
    return ISING_OK;
}

ising_status ising_prune_dev(ising_ctx *ctx, const ising_problem *problem, ising_pruned **out, void *stream) {
    if (!ctx || !out) return ISING_EINVAL;
    *out = nullptr;
    ST_TRY(check_problem_shape(ctx, problem));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Ingest ing;
    ST_TRY(ingest(ctx, to_dev(*problem), ctx->pool, ing, s));
    auto pr = std::make_unique<ising_pruned>();
    pr->device = ctx->device;
    pr->pool = &pr->own;
    ST_TRY(prune_core(ctx, to_dev(*problem), *pr, s));
    *out = pr.release();
    return ISING_OK;
}

void ising_pruned_free(ising_pruned *pruned) {
    if (!pruned) return;
    (void)hipSetDevice(pruned->device);
    (void)hipDeviceSynchronize();
    delete pruned;
}

ising_status ising_pruned_info(const ising_pruned *pr, int32_t *n, int32_t *n_G, int32_t *rounds, int64_t *nnz_G,
                               double *C) {
    if (!pr) return ISING_EINVAL;
    if (n) *n = pr->n;
    if (n_G) *n_G = pr->nG;
    if (rounds) *rounds = pr->rounds;
    if (nnz_G) *nnz_G = pr->nnzG;
    if (C) *C = pr->C;
    return ISING_OK;
}

ising_status ising_pruned_record_dev(ising_ctx *ctx, const ising_pruned *pr, int8_t *kind, int32_t *round_of,
                                     int8_t *fixed, int32_t *partner, int8_t *sigma, int32_t *G, void *h_G,
                                     void *stream) {
    if (!ctx || !pr) return ISING_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, launch_copy_record(pr->w, pr->n, kind, round_of, fixed, partner, sigma, s));
    if (G && pr->nG > 0) {
        if (pr->identity) {
            std::vector<int32_t> idx(pr->n);
            for (int i = 0; i < pr->n; ++i) idx[i] = i;
            HIP_TRY(ctx, hipMemcpyAsync(G, idx.data(), (size_t)pr->n * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(ctx, hipStreamSynchronize(s));
        } else {
            HIP_TRY(ctx, hipMemcpyAsync(G, pr->w.G, (size_t)pr->nG * 4, hipMemcpyDeviceToDevice, s));
        }
    }
    if (h_G && pr->nG > 0 && pr->reduced.h) {
        const size_t sz = pr->identity ? vsize(pr->vtype) : (pr->vtype == ISING_I32 ? 4 : 8);
        HIP_TRY(ctx, hipMemcpyAsync(h_G, pr->reduced.h, (size_t)pr->nG * sz, hipMemcpyDeviceToDevice, s));
    }
    return ISING_OK;
}

ising_status ising_pruned_problem(const ising_pruned *pr, ising_problem *reduced) {
    if (!pr || !reduced) return ISING_EINVAL;
    *reduced = pr->reduced;
    return ISING_OK;
}

ising_status ising_pruned_copy_dev(ising_ctx *ctx, const ising_pruned *pr, void *J_or_val, int32_t *row_ptr,
                                   int32_t *col, void *h, void *stream) {
    if (!ctx || !pr) return ISING_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const ising_problem &r = pr->reduced;
    if (r.n == 0) return ISING_OK;
    const size_t vs = vsize(r.value_type);
    if (r.format == ISING_DENSE) {
        if (J_or_val) HIP_TRY(ctx, hipMemcpyAsync(J_or_val, r.J, (size_t)r.n * r.n * vs, hipMemcpyDeviceToDevice, s));
    } else {
        if (row_ptr) HIP_TRY(ctx, hipMemcpyAsync(row_ptr, r.row_ptr, (size_t)(r.n + 1) * 4, hipMemcpyDeviceToDevice, s));
        if (col && r.nnz) HIP_TRY(ctx, hipMemcpyAsync(col, r.col, (size_t)r.nnz * 4, hipMemcpyDeviceToDevice, s));
        if (J_or_val && r.nnz) HIP_TRY(ctx, hipMemcpyAsync(J_or_val, r.val, (size_t)r.nnz * vs, hipMemcpyDeviceToDevice, s));
    }
    if (h && r.h) HIP_TRY(ctx, hipMemcpyAsync(h, r.h, (size_t)r.n * vs, hipMemcpyDeviceToDevice, s));
    return ISING_OK;
}

ising_status ising_unprune_dev(ising_ctx *ctx, const ising_pruned *pr, const int8_t *s_G, int8_t *s_out,
                               void *stream) {
    if (!ctx || !pr || !s_out || (pr->nG > 0 && !s_G)) return ISING_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (pr->identity) {
        HIP_TRY(ctx, hipMemcpyAsync(s_out, s_G, pr->n, hipMemcpyDeviceToDevice, s));
        return ISING_OK;
    }
    HIP_TRY(ctx, launch_unprune(pr->w, pr->n, pr->rounds, s_G, s_out, s));
    return ISING_OK;
}

int32_t ising_ds_max_n(int32_t precision) { return ds_max_n(precision == ISING_PREC_FP64); }

ising_status ising_ds_dev(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                          const void *uniform, int32_t t0, int32_t steps, ising_ds_state *state, void *stream) {
    if (!ctx || !params) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Ingest ing;
    ST_TRY(ingest(ctx, to_dev(*problem), ctx->pool, ing, s));
    return run_ds(ctx, *problem, *params, ing, uniform, t0, steps, state, ctx->pool, s);
}

ising_status ising_ds_dense_dev(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                                const void *uniform, int32_t t0, int32_t steps, ising_ds_state *state, void *stream) {
    if (!ctx || !params) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Ingest ing;
    ST_TRY(ingest(ctx, to_dev(*problem), ctx->pool, ing, s));
    return run_dense(ctx, *problem, *params, uniform, t0, steps, state, ctx->pool, s, dense_exact(ing, problem->n));
}

ising_status ising_select_dev(ising_ctx *ctx, const double *e_best, int32_t replicas, int32_t *best,
                              void *stream) {
    if (!ctx || !e_best || !best || replicas <= 0) return ISING_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_select(e_best, replicas, best, (hipStream_t)stream));
    return ISING_OK;
}

// Whole solve on device buffers.  Blocking (pruning reads a counter per round).
ising_status ising_solve_dev(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                             int8_t *spins_out, double *energy_out, int64_t *energy_int_out,
                             ising_stats *stats_out, void *stream) {
    if (!ctx || !params || !spins_out) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    if (params->replicas <= 0 || params->steps < 0) return fail(ctx, ISING_EINVAL, "bad replicas/steps");
    ST_TRY(check_params(ctx, *params));
    if (energy_int_out && problem->value_type != ISING_I32)
        return fail(ctx, ISING_EINVAL, "integer energies need an ISING_I32 problem");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Pool &pool = ctx->pool;
    hipEvent_t ev[7];
    for (auto &e : ev) HIP_TRY(ctx, hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int k = 0; k < 7; ++k) (void)hipEventDestroy(e[k]);
        }
    } guard{ev};
    const auto t_host0 = std::chrono::steady_clock::now();
    HIP_TRY(ctx, hipEventRecord(ev[0], s));
    const DevProblem dp = to_dev(*problem);
    Ingest ing;
    ST_TRY(ingest(ctx, dp, pool, ing, s));
    HIP_TRY(ctx, hipEventRecord(ev[1], s));

    ising_pruned pr;
    pr.device = ctx->device;
    pr.pool = &pool;
    const ising_problem *red = problem;
    if (params->prune) {
        ST_TRY(prune_core(ctx, dp, pr, s));
        red = &pr.reduced;
    } else {
        pr.n = pr.nG = problem->n;
        pr.identity = true;
        pr.rounds = 0;
    }
    HIP_TRY(ctx, hipEventRecord(ev[2], s));
    const int nG = red->n;
    const int R = params->replicas;
    const bool dense_engine = use_dense_engine(*red, *params);
    if (!dense_engine && (params->precision == ISING_PREC_BF16X2 || params->precision == ISING_PREC_BF16 ||
                          params->precision == ISING_PREC_FP8 || params->precision == ISING_PREC_I8X3 ||
                          params->precision == ISING_PREC_I8X2))
        return fail(ctx, ISING_ENOTSUP, "BF16, FP8 and INT8 forms need dense couplings");
    const size_t real = params->precision == ISING_PREC_FP64 ? 8 : 4;
    int32_t *bestdev = nullptr;
    int8_t *sG = nullptr;
    HIP_TRY(ctx, pool.get("solve.best", 8, (void **)&bestdev));
    HIP_TRY(ctx, pool.get("solve.sG", std::max(nG, 1), (void **)&sG));
    int32_t best_replica = -1, best_step = 0;
    std::vector<int32_t> conv_steps;
    if (nG > 0) {
        ising_ds_state st{};
        HIP_TRY(ctx, pool.get("solve.theta", (size_t)nG * R * real, &st.theta));
        if (params->optimizer == ISING_OPT_ADAM) {
            HIP_TRY(ctx, pool.get("solve.m", (size_t)nG * R * real, &st.m));
            HIP_TRY(ctx, pool.get("solve.v", (size_t)nG * R * real, &st.v));
        }
        HIP_TRY(ctx, pool.get("solve.sbest", (size_t)nG * R, (void **)&st.s_best));
        HIP_TRY(ctx, pool.get("solve.ebest", (size_t)R * 8, (void **)&st.e_best));
        HIP_TRY(ctx, pool.get("solve.bstep", (size_t)R * 4, (void **)&st.best_step));
        if (params->conv_tol > 0) HIP_TRY(ctx, pool.get("solve.conv", (size_t)R * 4, (void **)&st.conv_step));
        if (dense_engine)
            ST_TRY(run_dense(ctx, *red, *params, nullptr, 0, params->steps, &st, pool, s, dense_exact(ing, red->n),
                             ev[5], ev[6]));
        else ST_TRY(run_ds(ctx, *red, *params, ing, nullptr, 0, params->steps, &st, pool, s, ev[5], ev[6]));
        HIP_TRY(ctx, hipEventRecord(ev[3], s));
        HIP_TRY(ctx, launch_select(st.e_best, R, bestdev, s));
        HIP_TRY(ctx, launch_gather_row(st.s_best, nG, bestdev, sG, s));
        HIP_TRY(ctx, hipMemcpyAsync(&best_replica, bestdev, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        if (best_replica >= 0 && best_replica < R)
            HIP_TRY(ctx, hipMemcpyAsync(&best_step, st.best_step + best_replica, 4, hipMemcpyDeviceToHost, s));
        if (st.conv_step) {
            conv_steps.resize(R);
            HIP_TRY(ctx, hipMemcpyAsync(conv_steps.data(), st.conv_step, (size_t)R * 4, hipMemcpyDeviceToHost, s));
        }
    } else {
        HIP_TRY(ctx, hipEventRecord(ev[3], s));
    }
    if (pr.identity) {
        HIP_TRY(ctx, hipMemcpyAsync(spins_out, sG, problem->n, hipMemcpyDeviceToDevice, s));
    } else {
        HIP_TRY(ctx, launch_unprune(pr.w, pr.n, pr.rounds, sG, spins_out, s));
    }
    if (energy_out || energy_int_out) {
        void *partial = nullptr;
        HIP_TRY(ctx, pool.get("energy.partial", energy_partial_bytes(problem->n, 1), &partial));
        HIP_TRY(ctx, launch_energy(dp, spins_out, 1, partial, energy_out, energy_int_out, s));
    }
    HIP_TRY(ctx, hipEventRecord(ev[4], s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const double host_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
    if (stats_out) {
        ising_stats &o = *stats_out;
        std::memset(&o, 0, sizeof(o));
        o.n = problem->n;
        o.n_G = nG;
        o.rounds = pr.rounds;
        o.best_replica = best_replica;
        o.steps = params->steps;
        o.best_step = best_step;
        o.eta = 1.0 - (double)nG / problem->n;
        o.constant_C = params->prune ? pr.C : 0.0;
        o.t_upload_ms = ms_between(ev[0], ev[1]);
        o.t_prune_ms = ms_between(ev[1], ev[2]);
        o.t_ds_ms = ms_between(ev[2], ev[3]);
        o.t_finish_ms = ms_between(ev[3], ev[4]);
        o.t_total_ms = host_ms;
        o.t_ds_kernel_ms = nG > 0 ? ms_between(ev[5], ev[6]) : 0.0;
        o.replica_spin_updates_per_s =
            o.t_ds_ms > 0 ? (double)nG * R * params->steps / (o.t_ds_ms * 1e-3) : 0.0;
        o.mean_steps_run = params->steps;
        if (!conv_steps.empty()) {
            double sum = 0.0;
            for (int32_t c : conv_steps) {
                o.converged += c > 0;
                sum += c > 0 ? c : params->steps;
            }
            o.mean_steps_run = sum / R;
        }
    }
    return ISING_OK;
}

ising_status ising_solve(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                         int8_t *spins_out, double *energy_out, int64_t *energy_int_out, ising_stats *stats_out) {
    if (!ctx || !params || !spins_out) return ISING_EINVAL;
    ST_TRY(check_problem_shape(ctx, problem));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    Pool &pool = ctx->pool;
    const auto t0 = std::chrono::steady_clock::now();
    const int n = problem->n;
    ising_problem d;
    ST_TRY(upload_problem(ctx, *problem, pool, "in.", d, s));
    int8_t *sdev = nullptr;
    double *edev = nullptr;
    int64_t *eidev = nullptr;
    HIP_TRY(ctx, pool.get("out.s", n, (void **)&sdev));
    HIP_TRY(ctx, pool.get("out.E", 8, (void **)&edev));
    HIP_TRY(ctx, pool.get("out.Ei", 8, (void **)&eidev));
    const bool want_int = problem->value_type == ISING_I32;
    ST_TRY(ising_solve_dev(ctx, &d, params, sdev, edev, want_int ? eidev : nullptr, stats_out, s));
    HIP_TRY(ctx, hipMemcpyAsync(spins_out, sdev, n, hipMemcpyDeviceToHost, s));
    double e = 0;
    int64_t ei = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&e, edev, 8, hipMemcpyDeviceToHost, s));
    if (want_int) HIP_TRY(ctx, hipMemcpyAsync(&ei, eidev, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (energy_out) *energy_out = e;
    if (energy_int_out) *energy_int_out = want_int ? ei : 0;
    if (stats_out)
        stats_out->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return ISING_OK;
}

}  // extern "C"
