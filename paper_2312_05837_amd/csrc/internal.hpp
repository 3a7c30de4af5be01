// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "../../include/ising.h"

namespace ising {

// Device view of a problem (all pointers on the device).
struct DevProblem {
    int32_t n = 0;
    int32_t format = ISING_DENSE;
    int32_t vtype = ISING_I32;
    int64_t nnz = 0;
    const void *J = nullptr;
    const int32_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const void *val = nullptr;
    const void *h = nullptr;
};

inline DevProblem to_dev(const ising_problem &p) {
    DevProblem d;
    d.n = p.n;
    d.format = p.format;
    d.vtype = p.value_type;
    d.nnz = p.nnz;
    d.J = p.J;
    d.row_ptr = p.row_ptr;
    d.col = p.col;
    d.val = p.val;
    d.h = p.h;
    return d;
}

inline size_t vsize(int vtype) { return vtype == ISING_F64 ? 8 : 4; }

// ---- validation (kernels_validate.hip) -----------------------------------
// flags[0] bit 0: asymmetric, bit 1: nonzero diagonal, bit 2: bad CSR structure,
// bit 3: non-finite value.  flags[1]: max row degree.  flags[2]: 1 if every
// nonzero has the same magnitude.  flags[3]: 1 if every value of J and h is integral.
// wdev: one device double of scratch.  Synchronises the stream once.
hipError_t launch_validate(const DevProblem &p, int32_t *flags, double *wdev, hipStream_t s);
// Magnitude of the first stored nonzero coupling (1.0 if none), written to *w.
hipError_t launch_first_magnitude(const DevProblem &p, double *w, hipStream_t s);

// ---- energy (kernels_energy.hip) -----------------------------------------
// partial must hold energy_partial_bytes(n, count): count * ceil(n / 4) accumulators
// (int64 or double).
hipError_t launch_energy(const DevProblem &p, const int8_t *spins, int32_t count, void *partial,
                         double *E_out, int64_t *E_int_out, hipStream_t s);
size_t energy_partial_bytes(int32_t n, int32_t count);
// Size of the library's static device scratch for the energy partials (the entry point that
// allocates nothing), and its address on `device`, looked up once per device with that device
// current (the lookup is made by ising_create; later calls return the kept address).
constexpr size_t kEnergyScratchBytes = (size_t)8 << 20;
hipError_t energy_scratch_address(int device, void **ptr);

// ---- pruning (kernels_prune.hip) -------------------------------------------
struct PruneWork {
    int8_t *active, *isD, *isS, *cand;
    int8_t *kind, *fixed, *sigma;
    int32_t *round_of, *partner, *nb, *map, *G;
    void *h;        // working field: int64 (integer problems) or double
    void *jv;       // coupling to the unique neighbour: int64 or double
    void *cpart;    // per-spin contribution to C this phase
    void *C;        // accumulated constant (one int64 or double)
    // [0] = |D| this round, [1] = |S| this round, [2] = n_G, [3] = nnz_G, [4] = done (a round
    // removed nothing; later rounds return at once), [5] = rounds executed
    int32_t *counts;
};
hipError_t launch_prune_init(const DevProblem &p, const PruneWork &w, hipStream_t s);
hipError_t launch_prune_round(const DevProblem &p, const PruneWork &w, int32_t round, hipStream_t s);
hipError_t launch_prune_compact_scan(const DevProblem &p, const PruneWork &w, hipStream_t s);
// Reduced problem: dense J_G (n_G*n_G) or CSR (row_ptr_G filled by a scan, then cols/vals).
// Integer problems produce int32 values, real problems double values.
hipError_t launch_prune_gather_dense(const DevProblem &p, const PruneWork &w, int32_t nG, void *JG,
                                     void *hG, hipStream_t s);
hipError_t launch_prune_csr_count(const DevProblem &p, const PruneWork &w, int32_t nG,
                                  int32_t *row_ptr_G, hipStream_t s);
hipError_t launch_prune_csr_fill(const DevProblem &p, const PruneWork &w, int32_t nG,
                                 const int32_t *row_ptr_G, int32_t *col_G, void *val_G, void *hG,
                                 hipStream_t s);
hipError_t launch_unprune(const PruneWork &w, int32_t n, int32_t rounds, const int8_t *s_G,
                          int8_t *s_out, hipStream_t s);
hipError_t launch_copy_record(const PruneWork &w, int32_t n, int8_t *kind, int32_t *round_of,
                              int8_t *fixed, int32_t *partner, int8_t *sigma, hipStream_t s);

// ---- domain selection, persistent engine (kernels_ds.hip) -----------------
enum Coupling { CK_PM = 0, CK_CSRV = 1, CK_DENSE = 2, CK_PMS = 3 };

struct DSArgs {
    int32_t n = 0, R = 0, t0 = 0, steps = 0, opt = ISING_OPT_ADAM, init_mode = 0;
    uint64_t seed = 0;
    double lr = 6.0, mu = 0.5, b1 = 0.9, b2 = 0.999, eps = 1e-8;
    // coupling (device formats built by launch_ds_format)
    const int32_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const uint32_t *pm = nullptr;      // sign-packed entries: col | (J < 0) << 31
    // sign-packed entries in fixed-width rows for the wide engine (8+ spins per thread, degree
    // <= kEllWidth, block = launch bound of its spins per thread): [ept][block][kEllWidth words]
    // per position e * block + thread, the entries 2 col + (J < 0) of its neighbours (the byte of
    // the neighbour's term sgn(J) s in the vertex buffer; unused entries address the zero pair
    // 2 ept block); ellh: [ept][block] FP32, the position's field (0 without one or past n)
    const uint32_t *ell = nullptr;
    const float *ellh = nullptr;
    const void *val = nullptr;         // CSR values in the state precision
    const void *J = nullptr;           // dense values in the state precision
    double w = 1.0;                    // common magnitude of sign-packed couplings
    const void *h = nullptr;           // field in the state precision (nullable)
    // state
    void *theta = nullptr, *m = nullptr, *v = nullptr;
    const void *uniform = nullptr;
    int8_t *s_best = nullptr;
    double *e_best = nullptr;
    int32_t *best_step = nullptr;
    double *etrace = nullptr, *ltrace = nullptr;
    const void *bias = nullptr;        // 2*steps bias corrections (ADAM), state precision
    // staged +-w image (CK_PMS), indexed by thread-layout position q = e * block + thread
    const void *pimg = nullptr;        // groups of 4 uint16 byte offsets, group-major per wavefront
    int32_t pimg_groups = 0;
    const int32_t *prow = nullptr;     // group 0 of position q
    const uint32_t *pcnt = nullptr;    // degree | wavefront group count << 16
    const int32_t *pperm = nullptr;    // spin held at position q
    int32_t pms_rb = 0;                // bytes of one vertex region (pms_region_bytes)
    int32_t loss = ISING_LOSS_VERTEX;  // RELAXED: also z = J sin(theta) from an LDS copy of sin(theta)
    // nonzero: no field, and every coupling product and energy sum is an integer below 2^24 in the
    // state precision (integer w, w * nnz < 2^24), so sums may be taken in any order
    int32_t exact_sums = 0;
    // convergence test (off when conv_tol <= 0): each wavefront replays it on the step's losses
    double conv_tol = 0.0;
    int32_t conv_window = 5;
    int32_t *conv_step = nullptr;      // nullable: R steps at which the test held (0: never)
    // R * (kConvWindowMax + 1) values of the state precision: the last conv_window losses by
    // global step mod conv_window, then L_1; read when t0 > 0, written at the end of the call
    void *conv_state = nullptr;
};
constexpr int kConvWindowMax = 8;
constexpr int kEllWidth = 4;  // neighbour slots per fixed-width row, one 32-bit word each

struct DSLaunch {
    int coupling = CK_CSRV;
    bool fp64 = false;
    int rg = 1;      // replicas per workgroup
    int ept = 1;     // spins per thread
    int block = 64;  // threads per workgroup
    bool relaxed = false;  // relaxed-vertex loss: LDS holds sin(theta) too (not the streaming engine)
    bool conv = false;     // convergence test: LDS holds each wavefront's window of losses
};

// Build the engine's device formats: pm entries (if sign-packed), values and h
// converted to the state precision.  Buffers are caller-provided.
hipError_t launch_ds_format(const DevProblem &p, bool fp64, bool packed, uint32_t *pm, void *val_out,
                            void *h_out, hipStream_t s);
// kernel (nullable): receives the name of the kernel form that was launched.
hipError_t launch_ds(const DSArgs &a, const DSLaunch &l, hipStream_t s, std::string *kernel = nullptr);
// ADAM bias corrections 1/(1-b1^t), 1/(1-b2^t), t = t0+1..t0+steps (FP64, rounded).
hipError_t launch_bias_table(double b1, double b2, int t0, int steps, bool fp64, void *out, hipStream_t s);
int32_t ds_max_n(bool fp64);
// largest workgroup of the persistent engine with `ept` spins per thread (0: streaming)
int ds_block_limit(int ept);
// The fixed-width-row form for small problems: one replica per workgroup of kPmeSmallBlock
// threads with pme_small_ept(n) spins per thread (4 up to n = 1024, 8 up to 2048; 0 above).
constexpr int kPmeSmallBlock = 256;
int pme_small_ept(int n);
// Fixed-width neighbour rows (DSArgs::ell, DSArgs::ellh) from the sign-packed CSR; every
// degree <= kEllWidth, block = ds_block_limit(ept) (or kPmeSmallBlock with pme_small_ept(n)),
// ept * block < 32768.  hf: the field in FP32 (nullable).  ell: ept * block * kEllWidth words;
// hrow: ept * block floats.
hipError_t launch_ell_format(const DevProblem &p, const uint32_t *pm, const float *hf, int ept, int block,
                             uint32_t *ell, float *hrow, hipStream_t s);
// Build the CK_PMS image; writes the total group count to *total_groups (host,
// synchronises once).  img may be NULL to only count.
// Work buffers of the CK_PMS format: deg, pos (n); perm, prow, pcnt (ept * block);
// total (1); img (8 bytes per group, nullptr on the sizing pass).
struct PmsWork {
    int32_t *deg = nullptr, *pos = nullptr, *perm = nullptr, *prow = nullptr, *total = nullptr;
    uint32_t *pcnt = nullptr;
    uint16_t *img = nullptr;
};
int pms_region_bytes(const DSLaunch &l);
// Sizing pass (w.img == nullptr): layout tables and the group count (synchronises s).
// Fill pass: the image.
// wunit: couplings are integer multiples of it (at most kPmsMaxMult); a coupling of
// magnitude k wunit is staged k times.
constexpr int kPmsMaxMult = 4;
hipError_t launch_pms_format(const DevProblem &p, const DSLaunch &l, double wunit, PmsWork &w,
                             int32_t *total_groups, hipStream_t s);
// Dynamic LDS bytes of a launch.  twin: the fixed-width-row form, whose vertex buffers (each
// sign and its negation) are a static array of 2 twin_stride(ept, block) bytes besides these
size_t ds_lds_bytes(const DSLaunch &l, int n, int pimg_groups, bool twin = false);
// Batched persistent engine (FP32): workgroup b runs replica group map[b].y of
// descs[map[b].x]; all descriptors share the launch configuration l.
hipError_t launch_ds_batch(const DSArgs *descs, const int2 *map, int nwg, const DSLaunch &l, size_t lds,
                           hipStream_t s);

hipError_t launch_select(const double *e_best, int32_t R, int32_t *best, hipStream_t s);
// s_G = rows[best] of a replica-major int8 block (device-side gather).
hipError_t launch_gather_row(const int8_t *block, int32_t n, const int32_t *best, int8_t *out,
                             hipStream_t s);

// ---- domain selection for dense couplings on MFMA (kernels_dense.hip) --------
enum DenseForm { DF_FP32 = 0, DF_BF16X2 = 1, DF_BF16 = 2, DF_FP8 = 3, DF_I8X3 = 4, DF_I8X2 = 5, DF_I8X1 = 6 };

// Vertex buffers of the matrix-core engine: step t reads buffer (t - 1) % 3 and writes t % 3, so
// the vertex scored in step t - 1 stays intact while step t's tiles keep its best-vertex record.
constexpr int kDenseVertexBufs = 3;
struct DenseRun {
    int n = 0, R = 0, Mp = 0, Kp = 0, form = DF_BF16X2, opt = ISING_OPT_ADAM, t0 = 0, steps = 0, init_mode = 2;
    int reinit = 1;
    uint64_t seed = 0;
    double lr = 6.0, mu = 0.5, b1 = 0.9, b2 = 0.999, eps = 1e-8;
    float jscale = 1.f;  // FP8 form: the common magnitude w of the couplings (operand J / w)
    // INT8 forms: the matrix's scale, device memory written by launch_dense_prepare (float 2^e at
    // byte 16, the exponent e as int32 at byte 20 of kDenseScaleBytes)
    const void *jsc = nullptr;
    const void *Jhi = nullptr, *Jlo = nullptr, *Jf = nullptr;
    const float *h = nullptr;
    const void *uniform = nullptr;
    void *S = nullptr;  // kDenseVertexBufs vertex buffers [R][Kp] (FP32, BF16 bits, FP8 or INT8 bytes)
    float *theta = nullptr, *m = nullptr, *v = nullptr;
    float *Epart = nullptr, *Lpart = nullptr;  // [2][Mp / 128][R], by step parity
    double *e_best = nullptr;
    int32_t *best_step = nullptr;
    int8_t *s_best = nullptr;
    double *etrace = nullptr, *ltrace = nullptr;
    const float *bias = nullptr;  // ADAM bias corrections of steps t0+1.. (2 floats per step)
};
// Pad and split J (and convert h to float into hf when both are non-null).  INT8 forms: Jhi
// holds the digit planes [D][Mp][Kp] and jsc (kDenseScaleBytes of device memory) receives the
// scale, found on the device.
constexpr size_t kDenseScaleBytes = 32;
hipError_t launch_dense_prepare(const DevProblem &p, int form, int Mp, int Kp, void *Jhi, void *Jlo, void *Jf,
                                float *hf, void *jsc, hipStream_t s);
// vertex operand bytes per element of a form
constexpr size_t dense_vertex_bytes(int form) {
    return form == DF_FP32 ? 4 : (form == DF_BF16X2 || form == DF_BF16) ? 2 : 1;
}
// J operand bytes per padded element of a form (all planes)
constexpr size_t dense_j_bytes(int form) {
    return form == DF_FP32 ? 4 : form == DF_BF16X2 ? 4 : form == DF_BF16 ? 2 : form == DF_I8X3 ? 3 : form == DF_I8X2 ? 2 : 1;  // FP8, I8X1
}
// State initialisation (t0 = 0) or vertex re-derivation (t0 > 0) before a chunk.
hipError_t launch_dense_init(const DenseRun &d, hipStream_t s);
// Advance `count` problems of the same form by `steps` steps: one launch per step for the whole
// group (each step's tiles also keep the previous step's best vertices) and one for the last
// step's best vertices.  scratch: dense_group_scratch_bytes() of device memory.
hipError_t launch_dense_group(const DenseRun *const *runs, int count, int steps, void *scratch, hipStream_t s);
// The same in two parts, for callers that capture the kernels in a graph: the upload of the
// group's descriptors and work lists to scratch (host-synchronous), and the steps + 1 kernel
// launches alone (no copies or fills), which read everything per-problem from scratch.
struct DenseGroupShape {
    int form = DF_BF16X2, descs = 0, tiles = 0, quads = 0;
};
hipError_t dense_group_upload(const DenseRun *const *runs, int count, void *scratch, hipStream_t s,
                              DenseGroupShape *shape);
hipError_t dense_group_launch(const DenseGroupShape &shape, void *scratch, int steps, hipStream_t s);
size_t dense_group_scratch_bytes(const DenseRun *const *runs, int count);
// One problem: init + group of one.
hipError_t launch_dense_run(const DenseRun &d, void *scratch, hipStream_t s);

}  // namespace ising
