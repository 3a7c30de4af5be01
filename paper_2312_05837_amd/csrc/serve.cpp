// Serving loop: continuous batching of many solves on one GPU.
//
// A scheduler thread owns the device work.  Each iteration it
//   1. admits queued requests (first come, first served) while their device
//      footprint fits the memory budget and a slot is free: upload, ingest
//      checks, pruning, device formats and state buffers;
//   2. advances every resident request by one chunk of domain-selection steps:
//      all sparse requests that share a launch configuration run in ONE launch
//      of the persistent engine (one workgroup per request x replica group,
//      each reading its own descriptor), dense requests run the matrix-core
//      engine on a small pool of streams, so their work overlaps;
//   3. harvests the requests that finished all their steps (best replica,
//      retrieval, exact energy, download), frees their memory and wakes waiters;
// so requests arriving while others run are admitted as soon as memory and
// slots free up.  A request's arithmetic depends only on its own problem,
// parameters and step range, never on its neighbours in a batch, so its
// result is bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"

using namespace ising;
using namespace ising::rt;

namespace ising {
namespace rt {

namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum ReqState { Q_QUEUED, Q_RESIDENT, Q_DONE };

struct Request {
    uint64_t ticket = 0;
    ising_params prm{};
    // host copy of the problem
    ising_problem hp{};
    std::vector<char> J, val, h;
    std::vector<int32_t> row_ptr, col;
    // lifecycle
    ReqState state = Q_QUEUED;
    bool cancel = false;
    ising_status result = ISING_OK;
    std::string error;
    std::vector<int8_t> spins;
    double energy = 0.0;
    ising_stats stats{};
    double t_submit = 0, t_admit0 = 0, t_admit1 = 0, t_done = 0;
    size_t bytes = 0;
    // device side
    std::unique_ptr<Pool> pool;
    ising_problem dp{};
    std::unique_ptr<ising_pruned> pr;
    const ising_problem *red = nullptr;
    Ingest ing;
    bool dense = false;
    DSArgs args;   // persistent engine (sparse)
    DSPlan plan;
    DenseRun drun; // matrix-core engine (dense)
    ising_ds_state st{};
    int steps_done = 0;
    std::vector<int32_t> conv_steps;  // convergence test: per replica, the step at which it stopped
    int dense_stream = 0;
};

}  // namespace

struct Server {
    ising_ctx *ctx = nullptr;
    ising_serve_config cfg{};
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int waiters = 0;  // ising_wait calls inside the server (stop releases it only when none is)
    uint64_t next_ticket = 1;
    std::deque<Request *> queue;
    std::vector<Request *> resident;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    size_t bytes_in_use = 0;
    ising_serve_info info{};
    hipStream_t main = nullptr;
    std::vector<hipStream_t> dense;
    Pool batch;  // descriptor and work-map buffers of the batched launches
    // replayable launch sequences of the dense groups, by group key: valid while the group's
    // shape, step count and scratch buffer are unchanged (the kernels read everything else
    // from the descriptors uploaded before each replay)
    struct DenseGraph {
        DenseGroupShape shape;
        int steps = 0;
        void *scratch = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<std::string, DenseGraph> graphs;
    // failure handling tests only (environment ISING_SERVE_TEST_FAIL_DENSE_STEPS, read at start):
    // a dense group advancing this many steps in a chunk reports a launch failure instead of
    // launching (0: off)
    int test_fail_dense_steps = 0;
};

namespace {

// Device footprint of a request, counted before admission.
size_t footprint(const Request &q) {
    const size_t n = q.hp.n, R = q.prm.replicas;
    const size_t vs = vsize(q.hp.value_type);
    size_t b = 0;
    if (q.hp.format == ISING_DENSE) {
        // (K padded to 128 covers every form's padding; 4 bytes per element covers every
        // form's J and vertex operands)
        const size_t Mp = (n + 127) / 128 * 128, Kp = (n + 127) / 128 * 128;
        b += n * n * vs;                 // J
        b += Mp * Kp * 4 + kDenseScaleBytes;  // split, digit planes or FP32 operand
        b += kDenseVertexBufs * R * Kp * 4;  // vertex buffers
        b += 2 * (Mp / 128) * R * 8;     // energy partials, by step parity
    } else {
        b += (n + 1) * 4 + q.hp.nnz * (4 + vs);   // CSR
        b += q.hp.nnz * 8 + n * 24;               // device formats
    }
    b += n * vs + n * 64;                          // field, pruning work
    b += R * n * (3 * 4 + 1) + R * 16;             // theta, m, v, best vertex, energies
    b += 64 * 1024;                                // small buffers
    return b;
}

ising_status admit(Server &S, Request &q) {
    ising_ctx *ctx = S.ctx;
    hipStream_t s = S.main;
    q.pool.reset(new Pool());
    Pool &pool = *q.pool;
    const int n = q.hp.n;
    const size_t vs = vsize(q.hp.value_type);
    q.dp = q.hp;
    void *buf = nullptr;
    if (q.hp.format == ISING_DENSE) {
        HIP_TRY(ctx, pool.get("J", (size_t)n * n * vs, &buf));
        HIP_TRY(ctx, hipMemcpyAsync(buf, q.J.data(), (size_t)n * n * vs, hipMemcpyHostToDevice, s));
        q.dp.J = buf;
    } else {
        void *rp = nullptr, *c = nullptr, *v = nullptr;
        HIP_TRY(ctx, pool.get("rp", (size_t)(n + 1) * 4, &rp));
        HIP_TRY(ctx, pool.get("col", (size_t)std::max<int64_t>(q.hp.nnz, 1) * 4, &c));
        HIP_TRY(ctx, pool.get("val", (size_t)std::max<int64_t>(q.hp.nnz, 1) * vs, &v));
        HIP_TRY(ctx, hipMemcpyAsync(rp, q.row_ptr.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s));
        if (q.hp.nnz > 0) {
            HIP_TRY(ctx, hipMemcpyAsync(c, q.col.data(), (size_t)q.hp.nnz * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(ctx, hipMemcpyAsync(v, q.val.data(), (size_t)q.hp.nnz * vs, hipMemcpyHostToDevice, s));
        }
        q.dp.row_ptr = (const int32_t *)rp;
        q.dp.col = (const int32_t *)c;
        q.dp.val = v;
    }
    if (q.hp.h) {
        HIP_TRY(ctx, pool.get("h", (size_t)n * vs, &buf));
        HIP_TRY(ctx, hipMemcpyAsync(buf, q.h.data(), (size_t)n * vs, hipMemcpyHostToDevice, s));
        q.dp.h = buf;
    }
    ST_TRY(ingest(ctx, to_dev(q.dp), pool, q.ing, s));
    q.pr.reset(new ising_pruned());
    q.pr->device = ctx->device;
    q.pr->pool = &pool;
    if (q.prm.prune) {
        ST_TRY(prune_core(ctx, to_dev(q.dp), *q.pr, s));
        q.red = &q.pr->reduced;
    } else {
        q.pr->n = q.pr->nG = n;
        q.pr->identity = true;
        q.red = &q.dp;
    }
    const int nG = q.red->n, R = q.prm.replicas;
    if (nG == 0) {  // everything was fixed by pruning
        q.steps_done = q.prm.steps;
        return ISING_OK;
    }
    q.dense = use_dense_engine(*q.red, q.prm);
    if (!q.dense && q.prm.precision != ISING_PREC_FP32)
        return fail(ctx, ISING_ENOTSUP, "served requests off the matrix cores (sparse, or with the convergence test) run in FP32");
    HIP_TRY(ctx, pool.get("theta", (size_t)nG * R * 4, &q.st.theta));
    if (q.prm.optimizer == ISING_OPT_ADAM) {
        HIP_TRY(ctx, pool.get("m", (size_t)nG * R * 4, &q.st.m));
        HIP_TRY(ctx, pool.get("v", (size_t)nG * R * 4, &q.st.v));
    }
    HIP_TRY(ctx, pool.get("sbest", (size_t)nG * R, (void **)&q.st.s_best));
    HIP_TRY(ctx, pool.get("ebest", (size_t)R * 8, (void **)&q.st.e_best));
    HIP_TRY(ctx, pool.get("bstep", (size_t)R * 4, (void **)&q.st.best_step));
    if (q.dense) {
        ST_TRY(prepare_dense(ctx, *q.red, q.prm, pool, s, q.drun, dense_exact(q.ing, q.red->n)));
        DenseRun &d = q.drun;
        d.lr = q.prm.lr;
        d.mu = q.prm.mu;
        d.b1 = q.prm.beta1;
        d.b2 = q.prm.beta2;
        d.eps = q.prm.eps;
        d.theta = (float *)q.st.theta;
        d.m = (float *)q.st.m;
        d.v = (float *)q.st.v;
        d.e_best = q.st.e_best;
        d.best_step = q.st.best_step;
        d.s_best = q.st.s_best;
        if (q.prm.optimizer == ISING_OPT_ADAM && q.prm.steps > 0) {
            void *bias = nullptr;
            HIP_TRY(ctx, pool.get("dbias", (size_t)2 * q.prm.steps * 4, &bias));
            HIP_TRY(ctx, launch_bias_table(q.prm.beta1, q.prm.beta2, 0, q.prm.steps, false, bias, s));
            d.bias = (const float *)bias;
        }
    } else {
        ST_TRY(prepare_ds(ctx, *q.red, q.prm, q.ing, pool, s, q.args, q.plan, /*register_only=*/true,
                          /*batched=*/true));
        if (q.plan.l.ept > 4)  // the batched launches hold at most 4 spins per thread
            return fail(ctx, ISING_ENOTSUP, "served sparse problems need at most 4096 spins after pruning");
        q.args.theta = q.st.theta;
        q.args.m = q.st.m;
        q.args.v = q.st.v;
        q.args.s_best = q.st.s_best;
        q.args.e_best = q.st.e_best;
        q.args.best_step = q.st.best_step;
        if (q.prm.conv_tol > 0) {
            // the test's stop steps and window of losses, carried from chunk to chunk
            HIP_TRY(ctx, pool.get("convstep", (size_t)R * 4, (void **)&q.args.conv_step));
            HIP_TRY(ctx, pool.get("convstate", (size_t)R * (kConvWindowMax + 1) * 4, &q.args.conv_state));
        }
        if (q.prm.optimizer == ISING_OPT_ADAM && q.prm.steps > 0) {
            // bias corrections of every step of the request, indexed from its first step
            void *bias = nullptr;
            HIP_TRY(ctx, pool.get("bias", (size_t)2 * q.prm.steps * 4, &bias));
            HIP_TRY(ctx, launch_bias_table(q.prm.beta1, q.prm.beta2, 0, q.prm.steps, false, bias, s));
            q.args.bias = bias;
        }
    }
    if (q.prm.steps == 0) {
        // no step to run: the state is initialised as a call of zero steps initialises it (angles
        // from the draws, best energies +inf with the all +1 vertex), so that the harvest reads
        // the same records as the plain solve
        if (q.dense) {
            DenseRun d0 = q.drun;
            d0.t0 = 0;
            d0.steps = 0;
            d0.init_mode = 2;
            HIP_TRY(ctx, launch_dense_init(d0, s));
        } else {
            DSArgs a0 = q.args;
            a0.t0 = 0;
            a0.steps = 0;
            a0.init_mode = 2;
            HIP_TRY(ctx, launch_ds(a0, q.plan.l, s));
        }
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return ISING_OK;
}

ising_status finish(Server &S, Request &q) {
    ising_ctx *ctx = S.ctx;
    hipStream_t s = S.main;
    Pool &pool = *q.pool;
    const int n = q.hp.n, nG = q.red ? q.red->n : 0, R = q.prm.replicas;
    int8_t *sG = nullptr, *sfull = nullptr;
    int32_t *best = nullptr;
    void *E = nullptr, *Ei = nullptr, *partial = nullptr;
    HIP_TRY(ctx, pool.get("sG", std::max(nG, 1), (void **)&sG));
    HIP_TRY(ctx, pool.get("s", n, (void **)&sfull));
    HIP_TRY(ctx, pool.get("best", 8, (void **)&best));
    HIP_TRY(ctx, pool.get("E", 8, &E));
    HIP_TRY(ctx, pool.get("Ei", 8, &Ei));
    HIP_TRY(ctx, pool.get("partial", energy_partial_bytes(n, 1), &partial));
    int32_t best_h = -1, bstep = 0;
    if (nG > 0) {
        HIP_TRY(ctx, launch_select(q.st.e_best, R, best, s));
        HIP_TRY(ctx, launch_gather_row(q.st.s_best, nG, best, sG, s));
    }
    if (q.pr->identity) HIP_TRY(ctx, hipMemcpyAsync(sfull, sG, n, hipMemcpyDeviceToDevice, s));
    else HIP_TRY(ctx, launch_unprune(q.pr->w, q.pr->n, q.pr->rounds, sG, sfull, s));
    const bool integer = q.hp.value_type == ISING_I32;
    HIP_TRY(ctx, launch_energy(to_dev(q.dp), sfull, 1, partial, (double *)E, integer ? (int64_t *)Ei : nullptr, s));
    q.spins.resize(n);
    HIP_TRY(ctx, hipMemcpyAsync(q.spins.data(), sfull, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(&q.energy, E, 8, hipMemcpyDeviceToHost, s));
    if (nG > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(&best_h, best, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        HIP_TRY(ctx, hipMemcpyAsync(&bstep, q.st.best_step + best_h, 4, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));
    ising_stats &o = q.stats;
    std::memset(&o, 0, sizeof(o));
    o.n = n;
    o.n_G = nG;
    o.rounds = q.pr->rounds;
    o.best_replica = best_h;
    o.best_step = bstep;
    o.steps = q.prm.steps;
    o.eta = 1.0 - (double)nG / n;
    o.constant_C = q.prm.prune ? q.pr->C : 0.0;
    o.mean_steps_run = q.prm.steps;
    if (!q.conv_steps.empty()) {
        double sum = 0.0;
        for (int32_t c : q.conv_steps) {
            o.converged += c > 0;
            sum += c > 0 ? c : q.prm.steps;
        }
        o.mean_steps_run = sum / R;
    }
    return ISING_OK;
}

// Group key of the batched persistent launches.
using BatchKey = std::tuple<int, int, int, int>;  // coupling, rg, ept, block

void run_chunk(Server &S, std::vector<Request *> &live) {
    ising_ctx *ctx = S.ctx;
    const int K = std::max(1, S.cfg.chunk_steps);
    std::map<BatchKey, std::vector<Request *>> groups;
    // by form: every dense request of a form advances together (run and its request)
    std::map<int, std::vector<std::pair<DenseRun, Request *>>> dense;
    for (Request *q : live) {
        const int left = q->prm.steps - q->steps_done;
        if (left <= 0 || q->red == nullptr || q->red->n == 0) continue;
        const int k = std::min(K, left);
        if (q->dense) {
            DenseRun d = q->drun;
            d.t0 = q->steps_done;
            d.steps = k;
            d.init_mode = q->steps_done > 0 ? 0 : 2;
            if (d.bias) d.bias += (size_t)2 * q->steps_done;
            if (launch_dense_init(d, S.dense[0]) != hipSuccess) {
                q->result = ISING_EDEVICE;
                q->error = "matrix-core initialisation failed";
                continue;
            }
            dense[d.form].emplace_back(d, q);
        } else {
            const DSLaunch &l = q->plan.l;
            groups[BatchKey(l.coupling, l.rg, l.ept, l.block)].push_back(q);
        }
    }
    // dense groups: problems with fewer steps left than the chunk finish inside it; split
    // each form's group by step count so that one launch sequence fits every member
    for (auto &g : dense) {
        struct StepGroup {
            std::vector<const DenseRun *> runs;
            std::vector<Request *> reqs;
        };
        std::map<int, StepGroup> by_steps;
        for (const auto &dq : g.second) {
            StepGroup &sg = by_steps[dq.first.steps];
            sg.runs.push_back(&dq.first);
            sg.reqs.push_back(dq.second);
        }
        for (auto &bsg : by_steps) {
            const std::pair<const int, std::vector<const DenseRun *>> bs(bsg.first, bsg.second.runs);
            void *scratch = nullptr;
            char key[32];
            snprintf(key, sizeof key, "dg%d.%d", g.first, bs.first);
            const size_t bytes = dense_group_scratch_bytes(bs.second.data(), (int)bs.second.size());
            hipError_t e = S.batch.get(key, bytes, &scratch);
            if (e == hipSuccess && S.test_fail_dense_steps > 0 && bs.first == S.test_fail_dense_steps) {
                e = hipErrorLaunchFailure;
            } else if (e == hipSuccess && S.cfg.no_graphs) {
                e = launch_dense_group(bs.second.data(), (int)bs.second.size(), bs.first, scratch, S.dense[0]);
            } else if (e == hipSuccess) {
                DenseGroupShape shape;
                e = dense_group_upload(bs.second.data(), (int)bs.second.size(), scratch, S.dense[0], &shape);
                Server::DenseGraph &G = S.graphs[key];
                const bool same = G.exec && G.steps == bs.first && G.scratch == scratch && G.shape.form == shape.form &&
                                  G.shape.descs == shape.descs && G.shape.tiles == shape.tiles &&
                                  G.shape.quads == shape.quads;
                if (e == hipSuccess && !same) {
                    if (G.exec) (void)hipGraphExecDestroy(G.exec);
                    G = Server::DenseGraph();
                    hipGraph_t graph = nullptr;
                    e = hipStreamBeginCapture(S.dense[0], hipStreamCaptureModeThreadLocal);
                    if (e == hipSuccess) {
                        const hipError_t el = dense_group_launch(shape, scratch, bs.first, S.dense[0]);
                        const hipError_t ec = hipStreamEndCapture(S.dense[0], &graph);
                        e = el != hipSuccess ? el : ec;
                    }
                    if (e == hipSuccess) e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
                    if (graph) (void)hipGraphDestroy(graph);
                    if (e == hipSuccess) {
                        G.shape = shape;
                        G.steps = bs.first;
                        G.scratch = scratch;
                    } else {
                        G.exec = nullptr;
                    }
                }
                if (e == hipSuccess) e = hipGraphLaunch(G.exec, S.dense[0]);
            }
            if (e != hipSuccess) {
                // only this group's requests: the other groups' launches are independent
                for (Request *q : bsg.second.reqs) {
                    q->result = ISING_EDEVICE;
                    q->error = "matrix-core group launch failed";
                }
            }
            S.info.launches += 2 * bs.first;
        }
    }
    for (auto &g : groups) {
        std::vector<DSArgs> descs;
        std::vector<int2> map;
        size_t lds = 0;
        const DSLaunch &l0 = g.second.front()->plan.l;
        for (Request *q : g.second) {
            DSArgs a = q->args;
            const int k = std::min(K, q->prm.steps - q->steps_done);
            a.t0 = q->steps_done;
            a.steps = k;
            a.init_mode = q->steps_done > 0 ? 0 : 2;
            if (a.bias) a.bias = (const char *)a.bias + (size_t)2 * q->steps_done * 4;
            const int idx = (int)descs.size();
            descs.push_back(a);
            for (int gi = 0; gi < q->prm.replicas / l0.rg; ++gi) map.push_back(make_int2(idx, gi));
            lds = std::max(lds, ds_lds_bytes(l0, q->red->n, a.pimg_groups));
        }
        void *dd = nullptr, *dm = nullptr;
        char key[64];
        snprintf(key, sizeof key, "%d.%d.%d.%d", l0.coupling, l0.rg, l0.ept, l0.block);
        if (S.batch.get(std::string("d") + key, descs.size() * sizeof(DSArgs), &dd) != hipSuccess ||
            S.batch.get(std::string("m") + key, map.size() * sizeof(int2), &dm) != hipSuccess ||
            hipMemcpyAsync(dd, descs.data(), descs.size() * sizeof(DSArgs), hipMemcpyHostToDevice, S.main) !=
                hipSuccess ||
            hipMemcpyAsync(dm, map.data(), map.size() * sizeof(int2), hipMemcpyHostToDevice, S.main) != hipSuccess ||
            launch_ds_batch((const DSArgs *)dd, (const int2 *)dm, (int)map.size(), l0, lds, S.main) != hipSuccess) {
            for (Request *q : g.second) {
                q->result = ISING_EDEVICE;
                q->error = "batched launch failed";
            }
        }
        S.info.launches += 1;
    }
    (void)hipStreamSynchronize(S.main);
    for (hipStream_t s : S.dense) (void)hipStreamSynchronize(s);
    for (Request *q : live) {
        q->steps_done = std::min(q->prm.steps, q->steps_done + K);
        // a request whose replicas have all met the convergence test is finished
        if (q->args.conv_step && !q->dense && q->result == ISING_OK) {
            q->conv_steps.resize(q->prm.replicas);
            if (hipMemcpy(q->conv_steps.data(), q->args.conv_step, (size_t)q->prm.replicas * 4,
                          hipMemcpyDeviceToHost) == hipSuccess) {
                bool all = true;
                for (int32_t c : q->conv_steps) all = all && c > 0;
                if (all) q->steps_done = q->prm.steps;
            }
        }
    }
    S.info.chunks += 1;
    (void)ctx;
}

void release(Server &S, Request &q) {
    q.pr.reset();
    q.pool.reset();
    S.bytes_in_use -= q.bytes;
}

void loop(Server *Sp) {
    Server &S = *Sp;
    (void)hipSetDevice(S.ctx->device);
    for (;;) {
        std::vector<Request *> to_admit;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv_work.wait(lk, [&] { return S.stop || !S.queue.empty() || !S.resident.empty(); });
            if (S.stop && S.queue.empty() && S.resident.empty()) break;
            // admission: FIFO, by memory budget and slots
            while (!S.queue.empty()) {
                Request *q = S.queue.front();
                if (q->cancel) {
                    S.queue.pop_front();
                    q->result = ISING_ECANCELED;
                    q->state = Q_DONE;
                    q->t_done = now_ms();
                    S.info.canceled += 1;
                    S.cv_done.notify_all();
                    continue;
                }
                if ((int)(S.resident.size() + to_admit.size()) >= S.cfg.max_resident) break;
                const size_t need = footprint(*q);
                if (S.bytes_in_use + need > S.cfg.hbm_budget_bytes) {
                    if (S.resident.empty() && to_admit.empty()) {
                        S.queue.pop_front();
                        q->result = ISING_ENOMEM;
                        q->error = "request larger than the serving memory budget";
                        q->state = Q_DONE;
                        q->t_done = now_ms();
                        S.info.failed += 1;
                        S.cv_done.notify_all();
                        continue;
                    }
                    break;
                }
                S.queue.pop_front();
                q->bytes = need;
                S.bytes_in_use += need;
                to_admit.push_back(q);
            }
        }
        for (Request *q : to_admit) {
            q->t_admit0 = now_ms();
            ising_status st = admit(S, *q);
            q->t_admit1 = now_ms();
            std::lock_guard<std::mutex> lk(S.mu);
            if (st != ISING_OK) {
                q->result = st;
                q->error = error_copy(S.ctx);
                q->state = Q_DONE;
                q->t_done = now_ms();
                release(S, *q);
                S.info.failed += 1;
                S.cv_done.notify_all();
            } else {
                q->state = Q_RESIDENT;
                S.resident.push_back(q);
                S.info.admitted += 1;
            }
        }
        std::vector<Request *> live;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            live = S.resident;
        }
        if (live.empty()) continue;
        const double t0 = now_ms();
        run_chunk(S, live);
        S.info.busy_ms += now_ms() - t0;
        // harvest
        for (Request *q : live) {
            const bool done = q->steps_done >= q->prm.steps || q->result != ISING_OK || q->cancel;
            if (!done) continue;
            ising_status st = q->result;
            if (st == ISING_OK && q->cancel) st = ISING_ECANCELED;
            if (st == ISING_OK) st = finish(S, *q);
            std::lock_guard<std::mutex> lk(S.mu);
            q->result = st;
            if (st != ISING_OK && q->error.empty()) q->error = error_copy(S.ctx);
            q->t_done = now_ms();
            q->state = Q_DONE;
            S.resident.erase(std::find(S.resident.begin(), S.resident.end(), q));
            release(S, *q);
            if (st == ISING_OK) S.info.completed += 1;
            else if (st == ISING_ECANCELED) S.info.canceled += 1;
            else S.info.failed += 1;
            S.cv_done.notify_all();
        }
    }
}

}  // namespace
}  // namespace rt
}  // namespace ising

extern "C" {

ising_status ising_serve_start(ising_ctx *ctx, const ising_serve_config *cfg) {
    if (!ctx) return ISING_EINVAL;
    if (ctx->server) return fail(ctx, ISING_EBUSY, "a server is already running on this context");
    auto S = std::make_unique<Server>();
    S->ctx = ctx;
    ising_serve_config c{};
    c.hbm_budget_bytes = (size_t)16 << 30;
    c.max_resident = 64;
    c.chunk_steps = 100;
    c.dense_streams = 4;
    if (cfg) {
        if (cfg->hbm_budget_bytes) c.hbm_budget_bytes = cfg->hbm_budget_bytes;
        if (cfg->max_resident > 0) c.max_resident = cfg->max_resident;
        if (cfg->chunk_steps > 0) c.chunk_steps = cfg->chunk_steps;
        if (cfg->dense_streams > 0) c.dense_streams = cfg->dense_streams;
    }
    S->cfg = c;
    if (const char *f = std::getenv("ISING_SERVE_TEST_FAIL_DENSE_STEPS")) S->test_fail_dense_steps = std::atoi(f);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamCreateWithFlags(&S->main, hipStreamNonBlocking));
    S->dense.resize(c.dense_streams);
    for (auto &s : S->dense) HIP_TRY(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Server *raw = S.get();
    S->thr = std::thread(loop, raw);
    ctx->server = S.release();
    return ISING_OK;
}

ising_status ising_serve_stop(ising_ctx *ctx) {
    if (!ctx || !ctx->server) return ISING_EINVAL;
    Server *S = ctx->server;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->thr.joinable()) S->thr.join();
    {
        // every request is finished now; waits blocked on them return before the server goes
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->waiters == 0; });
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamDestroy(S->main);
    for (auto &g : S->graphs)
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
    for (auto s : S->dense) (void)hipStreamDestroy(s);
    S->batch.release();
    delete S;
    ctx->server = nullptr;
    return ISING_OK;
}

ising_status ising_submit(ising_ctx *ctx, const ising_problem *problem, const ising_params *params,
                          uint64_t *ticket) {
    if (!ctx || !params || !ticket) return ISING_EINVAL;
    Server *S = ctx->server;
    if (!S) return ISING_EINVAL;
    {
        // shape checks only; content checks run on the device at admission
        std::lock_guard<std::mutex> lk(S->mu);
        if (!problem || problem->n <= 0 || params->replicas <= 0 || params->steps < 0) return ISING_EINVAL;
    }
    if (problem->value_type < ISING_I32 || problem->value_type > ISING_F64) return ISING_EINVAL;
    if (check_params(nullptr, *params) != ISING_OK) return ISING_EINVAL;
    // the batched launches run the vertex loss (fixed step counts, or until the convergence test)
    if (params->loss != ISING_LOSS_VERTEX) return ISING_ENOTSUP;
    auto q = std::make_unique<Request>();
    q->prm = *params;
    q->hp = *problem;
    const size_t n = problem->n, vs = vsize(problem->value_type);
    if (problem->format == ISING_DENSE) {
        if (!problem->J) return ISING_EINVAL;
        q->J.assign((const char *)problem->J, (const char *)problem->J + n * n * vs);
    } else if (problem->format == ISING_CSR) {
        if (!problem->row_ptr || problem->nnz < 0 || (problem->nnz > 0 && (!problem->col || !problem->val)))
            return ISING_EINVAL;
        q->row_ptr.assign(problem->row_ptr, problem->row_ptr + n + 1);
        q->col.assign(problem->col, problem->col + problem->nnz);
        q->val.assign((const char *)problem->val, (const char *)problem->val + problem->nnz * vs);
    } else {
        return ISING_EINVAL;
    }
    if (problem->h) q->h.assign((const char *)problem->h, (const char *)problem->h + n * vs);
    q->hp.J = nullptr;
    q->hp.row_ptr = nullptr;
    q->hp.col = nullptr;
    q->hp.val = nullptr;
    q->hp.h = problem->h ? (const void *)1 : nullptr;  // marks "has a field"; the data is in q->h
    q->t_submit = now_ms();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return ISING_EBUSY;  // stopping: a request queued now would never run
    q->ticket = S->next_ticket++;
    *ticket = q->ticket;
    S->queue.push_back(q.get());
    S->all[q->ticket] = std::move(q);
    S->info.submitted += 1;
    S->cv_work.notify_all();
    return ISING_OK;
}

ising_status ising_wait(ising_ctx *ctx, uint64_t ticket, int32_t timeout_ms, int8_t *spins_out, double *energy_out,
                        ising_stats *stats_out) {
    if (!ctx || !ctx->server) return ISING_EINVAL;
    Server *S = ctx->server;
    std::unique_lock<std::mutex> lk(S->mu);
    // counted while inside (the guard is released before lk, so with the mutex held)
    struct Inside {
        Server *S;
        ~Inside() {
            --S->waiters;
            S->cv_done.notify_all();
        }
    } inside{S};
    ++S->waiters;
    if (S->all.find(ticket) == S->all.end()) return ISING_EINVAL;
    // the ticket is looked up again at every wake-up: another wait on it may have consumed it
    auto ready = [&] {
        auto i = S->all.find(ticket);
        return i == S->all.end() || i->second->state == Q_DONE;
    };
    if (timeout_ms < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return ISING_ETIMEDOUT;
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return ISING_EINVAL;  // consumed by another wait meanwhile
    Request *q = it->second.get();
    const ising_status st = q->result;
    if (st == ISING_OK) {
        if (spins_out) std::memcpy(spins_out, q->spins.data(), q->spins.size());
        if (energy_out) *energy_out = q->energy;
        if (stats_out) {
            *stats_out = q->stats;
            stats_out->t_upload_ms = (q->t_admit0 > 0 ? q->t_admit0 : q->t_done) - q->t_submit;  // queueing
            stats_out->t_prune_ms = q->t_admit1 - q->t_admit0;                                // admission
            stats_out->t_ds_ms = q->t_done - q->t_admit1;                                     // resident
            stats_out->t_total_ms = q->t_done - q->t_submit;                                  // latency
        }
    } else if (!q->error.empty()) {
        set_error(ctx, q->error);
    }
    S->all.erase(it);  // a ticket is consumed by its successful wait
    return st;
}

ising_status ising_cancel(ising_ctx *ctx, uint64_t ticket) {
    if (!ctx || !ctx->server) return ISING_EINVAL;
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return ISING_EINVAL;
    it->second->cancel = true;
    S->cv_work.notify_all();
    return ISING_OK;
}

ising_status ising_serve_query(ising_ctx *ctx, ising_serve_info *out) {
    if (!ctx || !ctx->server || !out) return ISING_EINVAL;
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->info;
    out->resident = (int32_t)S->resident.size();
    out->queued = (int32_t)S->queue.size();
    out->bytes_in_use = S->bytes_in_use;
    return ISING_OK;
}

}  // extern "C"
