/*
 * cutqc.h -- C ABI of the MI355X cut-circuit reconstruction library.
 *
 * The library reconstructs the output distribution of a quantum circuit that
 * has been cut into subcircuits (Tang & Martonosi, "Cutting Quantum Circuits
 * to Run on Quantum and Classical Platforms").  K wire cuts split an n-qubit
 * circuit into n_C subcircuits (Section 3.1).  Each subcircuit c is run in
 * every variant -- each downstream cut end initialised in |0>, |1>, |+> or
 * |+i>, each upstream cut end measured in the Z, X or Y basis -- and its
 * variant probabilities are turned into entry vectors E_c(l), one per Pauli
 * labelling l in {I,X,Y,Z} of the cuts it touches.  Eq. 1 then gives
 *
 *     p = 2^-K  sum over all 4^K labellings l  of  kron_c E_c(l restricted to c)
 *
 * (the printed Eq. 1 omits the 1/2 per cut of the Pauli decomposition; it is
 * applied here, once).  Full definition (Section 4.2) builds all 2^n values of
 * p; dynamic definition (Section 4.3, Algorithm 1) builds 2^{#active} bins per
 * recursion and zooms into the largest.
 *
 * Conventions (all entry points):
 *  - Subcircuit c has `width` register slots; slot 0 is the most significant
 *    bit of its outcome index.  init_cut[s] is the id of the cut whose
 *    downstream end initialises slot s, or -1; meas_cut[s] is the id of the
 *    cut whose upstream end is measured on slot s, or -1.  Slots with
 *    meas_cut == -1 are the subcircuit's outputs, n_c of them, in slot order.
 *    Cut ids are 0..K-1; each appears exactly once as init and once as meas,
 *    in two different subcircuits.
 *  - Label digits: I = 0, X = 1, Y = 2, Z = 3.  Row l of E_c is
 *    sum_j d_j 4^{k_c-1-j} over c's k_c cuts in ascending id order (the
 *    lowest id is the most significant digit).
 *  - Variant layout V_c[init][basis][outcome], row-major, shape
 *    (4^{r_c}, 3^{o_c}, 2^{w_c}): init digits |0>,|1>,|+>,|+i> = 0..3 over the
 *    init slots (slot order, first most significant), basis digits Z,X,Y =
 *    0..2 over the measured slots, then the register outcome.
 *  - Entry layout E_c[l][b], row-major (4^{k_c}, 2^{n_c}), b over c's outputs.
 *  - Output order: index = concatenation of b_0, b_1, ... with subcircuit 0
 *    most significant.  An optional out_perm[i] names the uncut qubit carried
 *    by concatenated bit i; the output is then in uncut-qubit order (qubit 0
 *    most significant).
 *
 * Memory and errors:
 *  - Pointers documented as "device" are HIP device memory owned by the
 *    caller; "host" arrays are read during the call only.  The library never
 *    allocates device memory: every intermediate lives in the caller's
 *    workspace, whose size the *_workspace_size queries return.
 *  - All arguments are validated before any launch; on error nothing is
 *    written and a status < 0 is returned (cq_last_error() has the detail).
 *    Nothing throws across the ABI and nothing aborts.
 *  - cq_attribute and cq_reconstruct_fd are asynchronous on `stream`, with
 *    one exception: the first cq_reconstruct_fd of a GEMM shape the autotuner
 *    has not seen (outside stream capture) times the kernel variants on
 *    `stream` and waits for them (see cq_autotune_enable; CQ_AUTOTUNE=0 or a
 *    warm-up call moves that cost out of a timed or captured region).
 *    cq_reconstruct_dd enqueues every recursion of the batch (by default as
 *    one captured graph), synchronises `stream` once at the end and returns
 *    after reading the records back.  Calls are thread-safe; calls that share
 *    a workspace must not overlap.
 */
#ifndef CUTQC_H
#define CUTQC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cq_status {
  CQ_OK = 0,
  CQ_ERR_ARG = -1,         /* null pointer, bad enum, bad count */
  CQ_ERR_SHAPE = -2,       /* sizes exceed the limits below */
  CQ_ERR_CUTMAP = -3,      /* inconsistent cut map */
  CQ_ERR_MASK = -4,        /* DD masks do not partition a subcircuit's outputs */
  CQ_ERR_WORKSPACE = -5,   /* workspace missing or too small */
  CQ_ERR_UNSUPPORTED = -6, /* valid but not supported by this build */
  CQ_ERR_HIP = -7          /* a HIP runtime call failed */
} cq_status;

/* Arithmetic of the label contractions.  Entries are always FP64 on input.
 * CQ_FP64: FP64 operands, FP64 matrix-core products, FP64 output.
 * CQ_FP32: FP32 operands, FP32 matrix-core products, FP32 output.
 * CQ_BF16 / CQ_FP16: 16-bit operands, FP32 accumulation, FP32 output.
 * CQ_BF16_SPLIT / CQ_FP16_SPLIT: each operand x = hi + lo with hi = rn16(x),
 *   lo = rn16(x - hi); products hi*hi + hi*lo + lo*hi, FP32 accumulation.
 * The FP16 forms scale every operand column by a power of two so that its
 * largest magnitude is near 1 and undo it in the FP32 epilogue (exact). */
typedef enum cq_precision {
  CQ_FP64 = 0,
  CQ_FP32 = 1,
  CQ_BF16 = 2,
  CQ_BF16_SPLIT = 3,
  CQ_FP16 = 4,
  CQ_FP16_SPLIT = 5
} cq_precision;

#define CQ_MAX_SUBCIRCUITS 8   /* the paper caps cut solutions at 5 (Section 4.1) */
#define CQ_MAX_CUTS 24         /* K */
#define CQ_MAX_LOCAL_CUTS 8    /* k_c: at most 4^8 label rows per subcircuit */
#define CQ_MAX_WIDTH 32        /* register slots per subcircuit */
#define CQ_MAX_FD_BITS 36      /* n for full definition (2^36 FP32 = 256 GiB) */
#define CQ_MAX_DD_ACTIVE 36    /* active qubits per DD recursion */
#define CQ_MAX_DD_R 16         /* DD recursions and list capacity */

typedef struct cq_subcircuit {
  int32_t width;            /* register slots w_c, 0..CQ_MAX_WIDTH */
  const int32_t* init_cut;  /* host, length width: cut id or -1 */
  const int32_t* meas_cut;  /* host, length width: cut id or -1 */
} cq_subcircuit;

/* Name of a status code (static string). */
const char* cq_status_string(cq_status s);

/* Detail of the last failing call on the calling thread (static per thread). */
const char* cq_last_error(void);

/* Host-only check of a cut map (no GPU needed).  Reports K and the total
 * number of outputs n when the pointers are non-null. */
cq_status cq_validate_cutmap(int32_t n_sub, const cq_subcircuit* subs, int32_t* n_cuts,
                             int32_t* n_outputs);

/* ---------------------------------------------------------------------------
 * Entry attribution (Section 3.1): variant probabilities -> entries.
 *
 *   E[l][b] = sum_j prod_t alpha(l_t, j_t)
 *             * sum_m prod_u sigma(l_u, m_u) * V[j][basis(l)][compose(b, m)]
 *
 * t over init slots, u over measured slots; alpha(I) = (1, 1, 0, 0),
 * alpha(X) = (-1, -1, 2, 0), alpha(Y) = (-1, -1, 0, 2), alpha(Z) = (1, -1, 0, 0)
 * over the prepared states |0>,|1>,|+>,|+i>; basis(I) = basis(Z) = Z,
 * basis(X) = X, basis(Y) = Y; sigma(I, m) = 1, otherwise (-1)^m.
 *
 * variants: device, FP64, layout V_c above.  entries: device, FP64, layout E_c
 * above (written whole).  workspace: device, at least
 * cq_attribute_workspace_size bytes (4^k_c * 2^n_c doubles).  FP64 throughout.
 * ------------------------------------------------------------------------- */
cq_status cq_attribute_workspace_size(const cq_subcircuit* sub, size_t* bytes);
cq_status cq_attribute(const cq_subcircuit* sub, const double* variants, double* entries,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Full-definition reconstruction (Eq. 1, Section 4.2).
 *
 * entries: host array of n_sub device pointers, FP64, layout E_c.
 * out: device, 2^n values, double when prec == CQ_FP64 else float, in
 *   concatenated order, or uncut-qubit order when out_perm (host, length n,
 *   a permutation of 0..n-1) is given.
 * The contraction runs as a sequence of label GEMMs on the matrix cores (the
 * shared cut labels are the reduction dimension); intermediates live in the
 * workspace (cq_fd_workspace_size bytes, which may be 0).
 * ------------------------------------------------------------------------- */
cq_status cq_fd_workspace_size(int32_t n_sub, const cq_subcircuit* subs, cq_precision prec,
                               const int32_t* out_perm, size_t* bytes);
cq_status cq_reconstruct_fd(int32_t n_sub, const cq_subcircuit* subs,
                            const double* const* entries, cq_precision prec,
                            const int32_t* out_perm, void* out, void* workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Full definition without allocation, for callers that cannot allocate device
 * memory: code under stream (graph) capture, tight serving loops, harnesses
 * that forbid allocation.
 *
 * Same arguments, kernels and results as cq_reconstruct_fd, minus the
 * workspace: the library keeps a fixed scratch array of
 * CQ_FD_NOALLOC_SCRATCH_BYTES in device memory on every GPU it runs this on
 * (held until the process ends; its device address is looked up on the first
 * call on each device).  A reconstruction whose workspace
 * (cq_fd_workspace_size) exceeds it is rejected with CQ_ERR_WORKSPACE before
 * any launch.  64 MiB covers the 20-qubit two-subcircuit workload (K = 4) in
 * every precision and chains of three 8-output subcircuits with K <= 6.
 * The call allocates nothing, creates no events and synchronises nothing (the
 * GEMM autotuner is not consulted beyond shapes it has already tuned; others
 * take the default kernel, which gives the same bits).  All calls on one GPU
 * share its scratch array, which keeps the last call's contents: calls that
 * overlap on one GPU (different streams, threads or graphs in flight) race.
 * ------------------------------------------------------------------------- */
#define CQ_FD_NOALLOC_SCRATCH_BYTES (64u << 20)

cq_status cq_reconstruct_fd_noalloc(int32_t n_sub, const cq_subcircuit* subs,
                                    const double* const* entries, cq_precision prec,
                                    const int32_t* out_perm, void* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Dynamic-definition reconstruction (Algorithm 1, Section 4.3).
 *
 * Masks are per subcircuit; bit i stands for output i of the subcircuit,
 * i = 0 being its most significant output.  active | merged | fixed must
 * partition the subcircuit's outputs; fixed_vals gives the zoomed values of
 * the fixed outputs (other bits must be 0).  Bins of a recursion are indexed
 * by the active outputs concatenated over subcircuits (subcircuit 0 most
 * significant, output order inside each), and bin v is the sum of p over all
 * states that agree with v on the active outputs, take the fixed values on
 * the fixed outputs and anything on the merged outputs.
 *
 * Per recursion the library: sums the entries over the merged outputs at the
 * fixed values (FP64); contracts the reduced entries in `prec` into the
 * 2^{#active} bins; when merged outputs remain, takes the 4R largest bins in
 * working precision, re-evaluates them in FP64 and appends the R largest to
 * the list L; sorts L (FP64 value descending, then recursion, then bin index),
 * keeps R entries and pops the head.  The popped bin's active outputs become
 * fixed at the bin's values and the first max_active[c] of its merged outputs
 * (output order) become active for the next recursion.  The run stops after R
 * recursions or when L is empty at a pop.
 *
 * Algorithm 1's state between two recursions -- the list L (each entry with
 * the masks of its bin), the next recursion index r and the masks to
 * reconstruct next -- can be saved after a call (params.checkpoint) and a
 * later call can continue from it (params.resume), so a run may be split
 * over several calls (params.recursions per call) and resumed after an
 * interruption.
 * ------------------------------------------------------------------------- */
typedef struct cq_dd_instance {
  int32_t n_sub;
  const cq_subcircuit* subs;     /* host, n_sub */
  const double* const* entries;  /* host array of n_sub device pointers, FP64, layout E_c */
  const uint64_t* active;        /* host, n_sub: recursion-0 masks */
  const uint64_t* merged;
  const uint64_t* fixed;
  const uint64_t* fixed_vals;
  const int32_t* max_active;     /* host, n_sub: outputs activated per zoom */
} cq_dd_instance;

typedef enum cq_dd_launch {
  CQ_DD_GRAPH = 0,   /* the whole batch captured into one hipGraph, launched once */
  CQ_DD_DIRECT = 1   /* the same launches issued directly on the stream */
} cq_dd_launch;

typedef struct cq_dd_params {
  cq_precision prec;  /* arithmetic of the bin contraction */
  int32_t R;          /* recursions and list capacity, 1..CQ_MAX_DD_R */
  int32_t launch;     /* cq_dd_launch */
  int32_t recursions; /* recursions this call runs per instance, counted from the state it
                         starts at; 0 or more than remain: up to recursion R - 1 */
  const void* resume; /* host, NULL or n_inst checkpoints (cq_dd_checkpoint_bytes each, as
                         written by an earlier call with the same instances, prec and R):
                         instance i continues from checkpoint i instead of its masks */
  void* checkpoint;   /* host, NULL or room for n_inst checkpoints: receives each instance's
                         state after the call */
} cq_dd_params;

/* Bytes of one instance's checkpoint (an opaque blob, valid for the library
 * build that wrote it). */
size_t cq_dd_checkpoint_bytes(void);

typedef struct cq_dd_record {  /* one recursion, written by the library */
  int32_t recursion;            /* its index r (0 for the first recursion of a fresh run) */
  uint64_t active[CQ_MAX_SUBCIRCUITS];
  uint64_t merged[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed[CQ_MAX_SUBCIRCUITS];
  uint64_t fixed_vals[CQ_MAX_SUBCIRCUITS];
  int32_t n_active;             /* log2 of the number of bins */
  double total;                 /* FP64 sum of all bins of the recursion */
  int32_t n_list;               /* entries of L after the update, before the pop */
  double list_val[CQ_MAX_DD_R]; /* FP64 values, sorted */
  int32_t list_rec[CQ_MAX_DD_R];
  uint64_t list_bin[CQ_MAX_DD_R];
  int32_t popped;               /* 1 when a bin was popped */
  int64_t tiles;                /* 128 x 128 output tiles of the contraction step that selects
                                   the candidate bins in its epilogue (0 when bins are stored) */
  int64_t tiles_run;            /* tile evaluations of that step: the warm-up tiles plus every
                                   tile whose bound reached the threshold (tile pruning skips
                                   the others) */
} cq_dd_record;

/* Workspace: a control block per instance (device program, recursion
 * state, launch descriptors, records) and the buffers of the recursions.
 * When no bins are stored (bins_stored == 0) and every instance's
 * contraction ends in a GEMM, so its bins never leave that GEMM's epilogue,
 * each instance has buffers of its own and instances with the same step
 * sequence advance in lockstep -- every kernel of a recursion is one launch
 * for all of them -- with such groups spread over up to 4 streams forked from
 * and joined back into `stream` (cq_dd_lanes).  Otherwise the instances share
 * the buffers of the largest and run one after another.  bins_stored != 0
 * when the caller passes a bin buffer for every recursion (then no bin
 * scratch is counted). */
cq_status cq_dd_workspace_size(int32_t n_inst, const cq_dd_instance* inst,
                               const cq_dd_params* params, int32_t bins_stored, size_t* bytes);

/* records: host, n_inst * R records (instance-major); the call's j-th
 * recursion of instance i (recursion r0 + j, r0 its starting index) goes to
 * records[i * R + j].  bins: NULL, or a host array of n_inst * R device
 * pointers indexed the same way, each NULL (bins go to workspace scratch) or
 * a buffer of 2^A values (double for CQ_FP64 else float), A = sum_c
 * max(#active_c at recursion 0, min(max_active[c], n_c)), the most bins a
 * recursion can have; the recursion's 2^n_active bins are written at its
 * start.  recursions_done: host, n_inst: recursions this call ran.  A resume
 * checkpoint that does not fit the instance (masks, list, index) is rejected
 * with CQ_ERR_ARG before any launch.
 *
 * Every recursion of every instance is enqueued without a host round trip:
 * shapes that depend on the zoom are computed on the device.  The call
 * returns after the records have been read back (it synchronises `stream`);
 * all validation happens before the first launch. */
cq_status cq_reconstruct_dd(int32_t n_inst, const cq_dd_instance* inst, const cq_dd_params* params,
                            cq_dd_record* records, void* const* bins, int32_t* recursions_done,
                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Breadth-first dynamic definition (Section 4.3: a breadth-first query that
 * refines a coarse picture of a dense distribution level by level).
 *
 * A node is one recursion of the root instance's circuit: its bins are
 * reconstructed as in cq_reconstruct_dd and its candidates are its `width`
 * largest bins (FP64-refined values) that still contain merged outputs,
 * value descending, then bin index ascending (node.rec.list_*, n_list of
 * them; list_rec is 0).  Level 0 is the root.  Level l + 1 has one node for
 * each of the `width` best candidates over all level-l nodes -- value
 * descending, then parent node ascending, then bin ascending -- zoomed as in
 * cq_reconstruct_dd: the bin's active outputs become fixed at its values and
 * the first max_active[c] merged outputs become active.  The query stops
 * after `levels` levels or at a level without candidates.  Each level runs
 * as one batched call (all its nodes captured together).
 * ------------------------------------------------------------------------- */
typedef struct cq_dd_bfs_params {
  cq_precision prec;  /* arithmetic of the bin contractions */
  int32_t levels;     /* >= 1 */
  int32_t width;      /* nodes per level and candidates per node, 1..CQ_MAX_DD_R */
  int32_t launch;     /* cq_dd_launch, per level */
} cq_dd_bfs_params;

typedef struct cq_dd_bfs_node {
  cq_dd_record rec;     /* the node's recursion: masks, n_active, total, candidates */
  int32_t level;
  int32_t parent;       /* index of the parent node in the output, -1 for the root */
  uint64_t parent_bin;  /* the parent's bin this node zooms into (0 for the root) */
} cq_dd_bfs_node;

/* Workspace for one level: `width` nodes planned like the root. */
cq_status cq_dd_bfs_workspace_size(const cq_dd_instance* root, const cq_dd_bfs_params* params,
                                   size_t* bytes);

/* root: as for cq_reconstruct_dd (entries stay on the device for the whole
 * query).  nodes: host, max_nodes >= 1 + (levels - 1) * width, filled in
 * level order; *n_nodes receives the count.  Validation of the root happens
 * before the first launch; each level is validated before its launches, so
 * an error at level l leaves the nodes of levels < l written.  Synchronises
 * `stream` once per level. */
cq_status cq_reconstruct_dd_bfs(const cq_dd_instance* root, const cq_dd_bfs_params* params,
                                cq_dd_bfs_node* nodes, int32_t max_nodes, int32_t* n_nodes,
                                void* workspace, size_t workspace_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Finite-shot emulation (Section 2: a QPU run reports the distribution of a
 * finite number of measured bit strings) and the chi-square loss (Eq. 3).
 *
 * Each row of a rows x cols FP64 probability table (one subcircuit variant's
 * 2^w outcomes, say) is sampled `shots` times, independently of the other
 * rows, and replaced by its empirical frequencies count / shots.  Every
 * decision is taken in integers, so the counts are a function of
 * (table, shots, seed) alone:
 *   q_i = floor(clamp(p_i, 0, 1) * 2^52), C_i = q_0 + ... + q_i (exact uint64);
 *   shot s of row r: Philox4x32-10 with key (seed & 0xffffffff, seed >> 32)
 *   and counter (s & 0xffffffff, s >> 32, r & 0xffffffff, r >> 32) gives words
 *   w0..w3; x = w0 + 2^32 w1; t = floor(x * T / 2^64) with T = C_{cols-1};
 *   the shot lands on the first i with C_i > t.
 * Negative entries count as zero probability; a row whose q sum to 0 gets no
 * counts (all frequencies 0).  Entries need not sum to 1: the row is sampled
 * in proportion to its clamped entries, whose sum must stay below 2^12 so
 * that C fits in 64 bits (a probability row sums to 1).  A row above that
 * is not detected: its counts are unspecified, but every access stays in
 * bounds.
 * ------------------------------------------------------------------------- */

/* Limits: 1 <= rows <= 65535, rows * cols <= 2^34, shots < 2^32,
 * rows * shots <= 2^34.  The workspace holds per-block sums and shot
 * counters of each row (2048 entries a block) and one 8-byte slot per shot. */
cq_status cq_sample_shots_workspace_size(int64_t rows, int64_t cols, int64_t shots, size_t* bytes);

/* probs: device, rows x cols row-major FP64, read only.  freqs: device,
 * rows x cols FP64, written (may not alias probs).  workspace: device, at
 * least cq_sample_shots_workspace_size bytes (prefix sums and counts),
 * owned by the caller, contents on entry ignored.  Asynchronous on `stream`;
 * arguments are checked before any launch (CQ_ERR_ARG, CQ_ERR_SHAPE,
 * CQ_ERR_WORKSPACE leave freqs untouched). */
cq_status cq_sample_shots(const double* probs, int64_t rows, int64_t cols, int64_t shots, uint64_t seed,
                          double* freqs, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Eq. 3: chi2 = sum_i (a_i - b_i)^2 / (a_i + b_i) over n entries; a term
 * with a_i + b_i = 0 contributes 0.  Applied as written to any real inputs,
 * so quasi-probabilities with negative entries can give negative terms.  The
 * sum runs in a fixed order (2048 x 256 threads summing four strided
 * streams each, then trees), so repeated calls give the same bits. */
cq_status cq_chi2_workspace_size(size_t* bytes);

/* a, b: device FP64, n >= 1 entries each.  result: device, one FP64,
 * written on `stream` (no synchronisation).  workspace: device, at least
 * cq_chi2_workspace_size bytes. */
cq_status cq_chi2(const double* a, const double* b, int64_t n, double* result, void* workspace,
                  size_t workspace_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * State-vector simulation on the device (the noiseless ground truth of
 * Section 2) and the variants of a subcircuit (Section 3.1), FP64 complex.
 *
 * A circuit is a list of gates on n qubits, qubit 0 the most significant bit
 * of a basis-state index: CQ_GATE_U applies the 2 x 2 unitary u (row-major,
 * (re, im) of u00, u01, u10, u11) to qubit q0; CQ_GATE_CZ applies CZ to q0
 * and q1.  The matrix is applied as given (unitarity is not checked).
 * Consecutive gates are applied in groups to tiles of 2^11 amplitudes held
 * in registers (8 per thread; registers narrower than a tile go through LDS),
 * in circuit order, so the state crosses HBM once per group.
 * ------------------------------------------------------------------------- */
#define CQ_MAX_SV_QUBITS 34  /* 2^34 amplitudes = 256 GiB of workspace */

typedef enum cq_gate_kind { CQ_GATE_U = 0, CQ_GATE_CZ = 1 } cq_gate_kind;

typedef struct cq_gate {
  int32_t kind;  /* cq_gate_kind */
  int32_t q0;    /* target qubit */
  int32_t q1;    /* second qubit of CQ_GATE_CZ, ignored otherwise */
  double u[8];   /* CQ_GATE_U matrix, ignored otherwise */
} cq_gate;

/* 16 * 2^n bytes (the state); n in 1..CQ_MAX_SV_QUBITS. */
cq_status cq_simulate_workspace_size(int32_t n, size_t* bytes);

/* |psi|^2 of gates applied to |0...0>.  gates: host, read during the call.
 * probs: device, 2^n FP64, written.  workspace: device, at least
 * cq_simulate_workspace_size bytes; it holds the state before the last
 * group of gates on return when there are two or more groups (the first
 * group generates |0...0> itself, so a single group leaves it unwritten).
 * Asynchronous on `stream`.  Errors (before any
 * launch): CQ_ERR_SHAPE for n out of range, CQ_ERR_ARG for a gate with an
 * unknown kind, a qubit out of range, equal CZ qubits or a non-finite
 * matrix entry, CQ_ERR_WORKSPACE. */
cq_status cq_simulate_probabilities(int32_t n, const cq_gate* gates, int32_t n_gates, double* probs,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream);

/* 16 * 2^width bytes per state.  Registers of at least 11 slots with at most
 * two measured ends hold several states at once: with one or two
 * initialised ends the 2^r computational init strings (every variant is a
 * combination of their results), else up to 16 init strings, within 4 GiB;
 * the size covers that many.  cq_variant_probabilities works with any
 * workspace of at least one state, more slowly below this size. */
cq_status cq_variants_workspace_size(const cq_subcircuit* sub, size_t* bytes);

/* Every variant of subcircuit `sub` running `gates` (qubits = its register
 * slots): for each init string (init slots in slot order, first most
 * significant, prepared in |0>, |1>, |+>, |+i> = digits 0..3; other slots
 * start in |0>) and each basis string (measured slots, Z, X, Y = digits
 * 0..2, rotated by nothing, H, or H S^dagger before the computational-basis
 * measurement), the probabilities of the 2^width register outcomes.
 * variants: device, FP64, layout (4^r, 3^o, 2^width) as cq_attribute reads
 * it, written whole.  workspace: device, at least one state (16 * 2^width
 * bytes); cq_variants_workspace_size bytes let it batch initial states.
 * Asynchronous on `stream`; errors as for cq_simulate_probabilities plus
 * the cut-map checks of the subcircuit. */
cq_status cq_variant_probabilities(const cq_subcircuit* sub, const cq_gate* gates, int32_t n_gates,
                                   double* variants, void* workspace, size_t workspace_bytes,
                                   hipStream_t stream);

/* -------------------------------------------------------------------------
 * Exact cut search for small circuits (Section 4.1; host only, no GPU).
 *
 * The circuit's two-qubit gates, in circuit order, are the vertices of its
 * DAG; each qubit wire joins consecutive two-qubit gates on that qubit
 * (one-qubit gates play no part).  A clustering of the gates into
 * subcircuits cuts every wire edge between two clusters.  Subcircuit c then
 * holds width_c qubits: the qubits whose first two-qubit gate it holds plus
 * one per cut it initialises; n_c = width_c minus the cuts it measures are
 * its outputs.  With the subcircuits ordered by n_c ascending, the cost is
 *     L = 4^K * sum_{c=2}^{n_C} prod_{i=1}^{c} 2^{n_i}
 * (the multiplications of Eq. 1's Kronecker products; 0 without cuts).
 * The search is exhaustive over clusterings into at most max_subcircuits
 * clusters with every width_c <= max_width, and returns the minimum; among
 * equal costs, the clustering whose label string (labels numbered in order
 * of first use) is lexicographically smallest.
 * ------------------------------------------------------------------------- */
#define CQ_MAX_FIND_GATES 16

typedef struct cq_cut_problem {
  int32_t n_qubits;            /* every qubit must take part in a two-qubit gate */
  int32_t n_gates;             /* two-qubit gates, 1..CQ_MAX_FIND_GATES */
  const int32_t* gate_qubits;  /* host, 2 * n_gates: the qubit pair of each gate */
  int32_t max_width;           /* qubits per subcircuit (the device size) */
  int32_t max_subcircuits;     /* 1..CQ_MAX_SUBCIRCUITS (the paper uses 5) */
} cq_cut_problem;

/* cluster: host, n_gates, receives each gate's subcircuit (0-based, numbered
 * in order of first use).  n_subcircuits, n_cuts, cost: host, receive n_C,
 * K and L.  Errors: CQ_ERR_ARG for null pointers, an empty circuit, gate
 * qubits out of range or equal, an idle qubit or limits out of range;
 * CQ_ERR_SHAPE for more than CQ_MAX_FIND_GATES gates or when no clustering
 * fits the limits.  Nothing is written on error. */
cq_status cq_find_cuts(const cq_cut_problem* problem, int32_t* cluster, int32_t* n_subcircuits,
                       int32_t* n_cuts, double* cost);

#ifdef __cplusplus
}
#endif

#endif /* CUTQC_H */
