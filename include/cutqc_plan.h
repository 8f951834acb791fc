/*
 * cutqc_plan.h -- host-only introspection of the contraction plan behind
 * cq_reconstruct_fd (and the bin contraction of cq_reconstruct_dd).
 *
 * Eq. 1 (Section 3.1) is evaluated as a sequence of batched label GEMMs
 *   C[z][m][n] = alpha * sum_k A[z*sAz + k*sAk + m] * B[z*sBz + k*sBk + n],
 *   stored at C[z*sCz + m*ldc + n],
 * and axis permutes dst[i] = alpha * src[sum_a idx_a(i) * sstride[a]], where
 * idx_a(i) are the digits of i in the mixed radix 2^log2[a] (last fastest).
 * This entry point reports that plan as JSON so tools and tests can inspect
 * or replay it without a GPU.  It launches nothing.
 */
#ifndef CUTQC_PLAN_H
#define CUTQC_PLAN_H

#include "cutqc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out_bits: host, n_sub, number of output bits each subcircuit contributes
 * (NULL: all of its outputs; the dynamic-definition bin contraction passes
 * the active counts).  out_perm as in cq_reconstruct_fd (NULL: none).
 * Writes a NUL-terminated JSON object into buf (host, buf_bytes) when it
 * fits and always sets *needed to the bytes required (including the NUL):
 *   {"workspace_bytes": W, "work_elem_bytes": 8|4, "flops": F,
 *    "tensors": [{"loc": "input"|"work"|"out", "index": i, "elems": n,
 *                 "offset": byte offset (work only)}, ...],
 *    "steps": [{"op": "gemm", "a", "b", "c", "Z", "M", "N", "K", "sAz", "sAk",
 *               "sBz", "sBk", "sCz", "ldc", "alpha"} |
 *              {"op": "permute", "src", "dst", "log2": [...], "sstride": [...],
 *               "alpha"}, ...]}
 * Returns CQ_ERR_ARG (with *needed set) when buf is too small. */
cq_status cq_plan_json(int32_t n_sub, const cq_subcircuit* subs, cq_precision prec,
                       const int32_t* out_bits, const int32_t* out_perm, char* buf,
                       size_t buf_bytes, size_t* needed);

/* Per-launch timing for tools and benchmarks.  While enabled (on != 0) every
 * kernel the library enqueues is bracketed by two HIP events recorded on the
 * caller's stream; the events add a few microseconds per launch and change
 * nothing else.  Process-wide switch. */
cq_status cq_profile_enable(int32_t on);

/* Waits for the recorded events, then writes up to `cap` records in launch
 * order -- kernel name (NUL-terminated, at most 31 characters), elapsed
 * milliseconds, and algorithmic floating-point operations of the launch
 * (0 when not a contraction) -- and clears them.  names: host, cap * 32 bytes;
 * ms, flops: host, cap entries each.  *count = records that were pending. */
cq_status cq_profile_read(char* names, double* ms, double* flops, int32_t cap, int32_t* count);

/* GEMM autotuner for the full-definition label GEMMs.  The first launch of
 * each GEMM shape (outside stream capture, at least 64 output tiles) times
 * every kernel variant twice on the caller's stream and keeps the fastest for
 * that shape; that call synchronises the stream.  Under stream capture a
 * shape tuned before keeps its variant and an untuned shape takes variant 0
 * (nothing is timed).  Variant v: bit 0 flips the tile raster order (M- or
 * N-fastest); v >> 1 picks, for the 16-bit forms, the asynchronous
 * LDS-staged kernel with its default ring depth (0), with the other depth
 * (1), the register-path kernel (2), the persistent kernel (3) or the
 * occupancy kernel with four (4) or three (5) resident workgroups per compute
 * unit; for FP32 the tiled kernel (0) or the persistent kernel (3).  FP64 has
 * variants 0 and 1; FP32 0, 1, 6 and 7 (6 and 7 where rows are 16-byte
 * aligned); 16-bit forms 0..11 (2..11 only where the asynchronous kernel's
 * alignment holds, 6..11 only without output exponents).  Every variant
 * computes the same sums.
 *
 * mode: 0 = variant 0 always (cached choices ignored); 1 = tune (the
 * default, also set by the environment variable CQ_AUTOTUNE unless it starts
 * with '0'); 2 + v = variant v always where it applies, else 0 (for tests).
 * Negative modes act as 0.  Process-wide; the cache is guarded by a mutex.
 * Always returns CQ_OK. */
cq_status cq_autotune_enable(int32_t mode);

/* Per-label balance of the 16-bit operands of cq_reconstruct_fd (Eq. 1's
 * labelling terms pair each cut's measured end with its initialised end, so
 * a power of two s_j(d) on every entry row whose digit at cut j is d on the
 * measuring subcircuit, and 1/s_j(d) on the initialising one, changes no
 * term): s_j(d) brings the largest magnitudes of the two sides within a
 * factor of two of each other before the 16-bit conversion.  FP16's narrow
 * exponent range is what it protects; for the BF16 forms (FP32's exponent
 * range) a power of two changes no rounding while every value stays in the
 * normal range, so their results are the same bit for bit with or without it
 * (only values near 2^-126 can round differently).  mode: 0 = off, 1 = FP16
 * and FP16-split (the default), 2 = every 16-bit form.  Process-wide.
 * Always CQ_OK. */
cq_status cq_label_balance_enable(int32_t mode);

/* Column scaling of the FP16 and FP16-split operands of cq_reconstruct_fd
 * and cq_reconstruct_dd (Eq. 1 is linear in each subcircuit's entry and an
 * output bin takes one column of every entry, so a power of two per column,
 * undone on the output, changes no term): every entry column is scaled by
 * the power of two that brings its largest magnitude into [0.5, 1) before
 * the conversion, and the contraction writing the output adds the exponents
 * back (on the dynamic-definition path, before the top-C comparison and in
 * its tile bounds).  It keeps bins that are tiny beside the largest ones
 * accurate relative to their own size; a dynamic-definition plan whose last
 * step is not a contraction writing the bins runs unscaled.  on: 1 (the
 * default) or 0.  Process-wide; it changes what cq_fd_workspace_size and
 * cq_dd_workspace_size report, so query the size after setting it.
 * Always CQ_OK. */
cq_status cq_column_scaling_enable(int32_t on);

/* Parallel lanes of cq_reconstruct_dd (instances whose bins stay inside
 * the contraction run on up to this many streams forked from the caller's,
 * each with its own copy of the per-instance buffers).  lanes <= 0 restores
 * the default (4); larger values are capped at 8.  Process-wide; it changes
 * what cq_dd_workspace_size reports, so query the size after setting it.
 * Always CQ_OK. */
cq_status cq_dd_lanes(int32_t lanes);

/* Tuned choices kept across processes.  cq_autotune_save writes every cached
 * choice to `path` (text, one shape per line, tagged with the kind of device
 * -- architecture and compute-unit count -- it was timed on);
 * cq_autotune_load adds the choices in `path` made on this kind of device to
 * the cache (shapes cached already keep their choice; lines it does not
 * recognise are skipped), so a caller that captures before its first eager
 * call still launches tuned variants.  The environment variable
 * CQ_TUNE_CACHE names a file that is loaded at the first tuned launch and
 * extended with every shape tuned afterwards.  CQ_ERR_ARG when the file
 * cannot be read or written. */
cq_status cq_autotune_load(const char* path);
cq_status cq_autotune_save(const char* path);

/* The cached choices as JSON:
 *   [{"prec": ..., "M", "N", "K", "Z", "variant": v,
 *     "schedule": {"kernel": "tiled" | "async" | "register" | "persistent" |
 *                  "occupancy", "tile": [128, 128], "ring": operand stages in
 *                  LDS (0: none), "workgroups_per_cu": resident workgroups the
 *                  kernel is built for (0: as many as fit), "raster": "default"
 *                  | "flipped"},
 *     "ms": [[v, ms], ...]}, ...]
 * *needed receives the length including the terminating NUL; with buf null
 * or buf_bytes below it, nothing is written and CQ_ERR_ARG is returned. */
cq_status cq_autotune_json(char* buf, size_t buf_bytes, size_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* CUTQC_PLAN_H */
