/*
 * ipcomp.h -- C ABI of the IPComp hot path on MI355X (gfx950).
 *
 * IPComp (arXiv 2502.04093) is an interpolation-based progressive lossy
 * compressor.  Compression predicts every point from already reconstructed
 * coarser points, level by level and one dimension at a time (Sec. 4.1,
 * Eq. interp-linear / Eq. interp-cubic), quantizes the residual within an
 * absolute error bound (Sec. 4.2.2), and stores the integer codes as
 * negabinary, prefix-XOR-coded bitplanes (Sec. 4.3-4.4).  Retrieval loads only
 * the planes a planner selects for an error bound or a bitrate (Sec. 5) and
 * reconstructs in one pass (Alg. 1); refinement adds planes to a resident
 * reconstruction (Alg. 2).  The statement of the problem (Sec. 3.1.2): a user
 * retrieves at fidelity F1 and refines to F2..Fn, and every retrieval meets its
 * error bound.
 *
 * Conventions for every call:
 *  - Device pointers are HIP device allocations on the context's device.
 *  - Calls are ordered on the context's hipStream and return when their
 *    results are ready (they synchronize that stream).
 *  - A context is not thread-safe; use one per host thread.
 *  - Errors are reported by status codes only.  On error every output pointer
 *    is set to NULL, nothing leaks, and ipc_last_error() holds a message.
 *  - Streams and states are owned by the library and released with their
 *    *_free call; a stream must outlive the states made from it, and a
 *    context must outlive the streams and states it made.
 */
#ifndef IPCOMP_H
#define IPCOMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IPC_OK = 0,
  IPC_EINVAL = -1,       /* invalid argument */
  IPC_ENOMEM = -2,       /* device or host allocation failed */
  IPC_ECORRUPT = -3,     /* serialized stream fails validation */
  IPC_EHIP = -4,         /* HIP runtime error */
  IPC_ESTATE = -5,       /* object used with the wrong context or stream */
  IPC_EUNSUPPORTED = -6  /* valid request outside what the library supports */
} ipc_status;

typedef enum { IPC_F32 = 0, IPC_F64 = 1 } ipc_dtype;
typedef enum { IPC_LINEAR = 0, IPC_CUBIC = 1 } ipc_interp;
typedef enum { IPC_TARGET_EB = 0, IPC_TARGET_BITRATE = 1 } ipc_target_kind;
/* Or-ed into ipc_target.kind: plan with the paper's plane groups per level
 * (Sec. 4.3: every pass of a level discards the same number of planes) instead
 * of per pass.  The bound reported is the same per-pass bound (Thm. 1 read per
 * pass); only the set of plans the planner chooses from is smaller. */
#define IPC_TARGET_LEVEL_GROUPS 0x100

/* Retrieval target (Sec. 5): an absolute L-infinity error bound, or a bitrate
 * in bits per value (the loaded bytes are at most bitrate * n / 8). */
typedef struct {
  int32_t kind;  /* ipc_target_kind, optionally | IPC_TARGET_LEVEL_GROUPS */
  double value;  /* > 0 */
} ipc_target;

/* Delta-y table of Thm. 1 (ipc_options.errq_mode):
 *   IPC_ERRQ_EXACT: per pass, the largest |q - q'_b| over the pass's codes
 *     (measured during compression);
 *   IPC_ERRQ_BOUND: the same for every pass, fixed before compression: the
 *     largest change discarding b negabinary digits can make to any code, the
 *     truncation uncertainty of Sec. 4.4.2 (floor((2^(b+1) - 1) / 3)).  Plans
 *     then load at least as much as with the exact table. */
#define IPC_ERRQ_EXACT 0
#define IPC_ERRQ_BOUND 1
/* Lossless stage of the stored planes (ipc_options.lossless; Sec. 6 runs a
 * general-purpose compressor there): IPC_LOSSLESS_ZWE keeps the blocks raw
 * (all-zero planes of a chunk are not stored), IPC_LOSSLESS_CODED also
 * entropy-codes them at the end of compression (ipc_stream_entropy_code). */
#define IPC_LOSSLESS_ZWE 0
#define IPC_LOSSLESS_CODED 1
/* ipc_options.debug_flags: IPC_DEBUG_PER_PASS compresses with the
 * one-pass-per-launch kernels where the fused level kernels would run (same
 * stream, a cross-check); IPC_DEBUG_VERIFY retrieves the new stream at full
 * precision and checks |x - x^| <= abs_eb at every point (exact bits for
 * values that are not finite), failing with IPC_ECORRUPT otherwise. */
#define IPC_DEBUG_PER_PASS 1u
#define IPC_DEBUG_VERIFY 2u

/* Compression options; pass NULL for the defaults {IPC_CUBIC,
 * nonprog_levels 0, default chunk shape, IPC_ERRQ_EXACT, IPC_LOSSLESS_ZWE,
 * no debug flags}.  Unknown modes or flags are rejected with IPC_EINVAL. */
typedef struct {
  int32_t interp;          /* ipc_interp */
  int32_t nonprog_levels;  /* top levels always fully loaded (L_p of Alg. 1) */
  uint8_t chunk_log2[3];   /* chunk extents (log2) per dimension; all 0 = default */
  uint8_t errq_mode;       /* IPC_ERRQ_* */
  uint8_t lossless;        /* IPC_LOSSLESS_* */
  uint8_t reserved[3];     /* 0 */
  uint32_t debug_flags;    /* IPC_DEBUG_* */
} ipc_options;

#define IPC_FLAG_CLAMPED_TO_EB 1u      /* E below the compression bound: full load */
#define IPC_FLAG_BUDGET_BELOW_MIN 2u   /* bitrate below the fixed bytes: coarsest plan */
#define IPC_FLAG_NOOP 4u               /* refine target already met: nothing loaded */
#define IPC_MAX_PASSES 100

/* What a retrieval or refinement did. */
typedef struct {
  double bound;               /* guaranteed max |x - x~| of the result */
  uint64_t bytes_loaded;      /* stream bytes the plan uses (fixed part included) */
  uint64_t bytes_total;       /* serialized stream size */
  uint64_t bytes_read;        /* plane bytes read by this call */
  uint32_t n_passes;
  uint32_t flags;             /* IPC_FLAG_* */
  uint8_t plan[IPC_MAX_PASSES]; /* planes discarded per pass (0 = all loaded) */
  float t_plan_ms;            /* host planner time */
  float t_device_ms;          /* device time of the call's kernels */
} ipc_info;

typedef struct ipc_ctx ipc_ctx;
typedef struct ipc_stream ipc_stream;
typedef struct ipc_state ipc_state;

/* Context on HIP device `device`, issuing work on `hip_stream` (a
 * hipStream_t; NULL = a stream the context creates and owns).  The owned
 * stream is a blocking stream, so HIP orders each of its operations after the
 * work queued on the null stream before it (and later null-stream work after
 * it): a field written by a pending null-stream kernel is complete before a
 * call reads it, and an output buffer is not written while earlier
 * null-stream work still uses it. */
ipc_status ipc_ctx_create(int device, void *hip_stream, ipc_ctx **out);
void ipc_ctx_destroy(ipc_ctx *ctx);
/* Switch the hipStream later calls are ordered on (NULL = the owned one). */
ipc_status ipc_ctx_set_stream(ipc_ctx *ctx, void *hip_stream);

/* Compress a C-ordered field (dims[0] slowest, ndim 1..3, every dim >= 1) of
 * float32 or float64 on the device with absolute error bound abs_eb > 0
 * (finite).  The field is read only and must stay valid for the call.
 * Every reconstructed value satisfies |x - x^| <= abs_eb (Sec. 4.2.2).
 * The returned stream is device resident.  On return every read of the field
 * is done; the stream's outlier index may still be building on the context's
 * stream, behind which every later call on the context is ordered. */
ipc_status ipc_compress(ipc_ctx *ctx, const void *field_dev, const uint64_t *dims, int ndim,
                        int dtype, double abs_eb, const ipc_options *opts, ipc_stream **out);

/* What a stream reconstructs (the field of the problem statement, Sec.
 * 3.1.2) and how it was compressed. */
typedef struct {
  int32_t ndim;            /* 1..3 */
  int32_t dtype;           /* ipc_dtype */
  uint64_t dims[3];        /* C order, dims[0] slowest; the first ndim used */
  int32_t interp;          /* ipc_interp */
  int32_t nonprog_levels;  /* top levels always fully loaded (L_p of Alg. 1) */
  double abs_eb;           /* compression bound (Sec. 4.2.2) */
  uint32_t n_passes;       /* anchors + one per level and dimension */
  int32_t coding;          /* 0 raw blocks, 1 entropy-coded blocks */
} ipc_stream_desc;
/* Fill `out` from the stream's header; IPC_EINVAL on a null argument. */
ipc_status ipc_stream_describe(const ipc_stream *s, ipc_stream_desc *out);

/* Serialized size of a stream in bytes (the compressed size). */
ipc_status ipc_stream_size(const ipc_stream *s, uint64_t *bytes);
/* Write the serialized stream -- the independent blocks of Fig.
 * overall-design, one per bitplane of each chunk, after the fixed tables -- to
 * host memory `dst` of `capacity` bytes (at least ipc_stream_size).
 * IPC_EINVAL when it is smaller. */
ipc_status ipc_stream_to_host(ipc_ctx *ctx, const ipc_stream *s, void *dst, uint64_t capacity);
/* Make a stream from serialized bytes (validated: IPC_ECORRUPT on any
 * inconsistency, IPC_EUNSUPPORTED for a chunk shape the kernels do not take;
 * `src` is only read during the call).  Tables, masks and outliers always go
 * to the device.  device_resident = 1: the bitplanes too.  device_resident =
 * 0: the bitplanes stay in pinned host memory that the kernels read in place,
 * so a retrieval or refinement moves only the planes its plan loads across
 * the host link (the progressive retrieval of Sec. 3.1.2 from a store that
 * keeps the whole stream; slower than device-resident planes). */
ipc_status ipc_stream_from_host(ipc_ctx *ctx, const void *src, uint64_t bytes, int device_resident,
                                ipc_stream **out);
void ipc_stream_free(ipc_stream *s);

/* Entropy stage for the stored bitplane blocks (stands in for the paper's
 * general-purpose lossless compressor, Sec. 6 setup).  Codes every stored
 * block -- one bitplane of one chunk -- on the device with an adaptive binary
 * range coder, one block per thread; a block is kept raw when its code is not
 * shorter.  Afterwards:
 *   - ipc_stream_size / ipc_stream_to_host give the coded serialized form
 *     (header byte 11 = 1, a byte per block with its stored words, then the
 *     stored blocks);
 *   - the planner charges every plane the bytes its blocks occupy in that
 *     form, so bitrate targets and ipc_info.bytes_loaded / bytes_read count
 *     coded bytes;
 *   - retrieval and refinement read the resident raw planes, unchanged.
 * A stream already coded is left as it is.  ipc_stream_from_host accepts both
 * forms and decodes a coded one on the device.  The coded payload stays on the
 * device beside the raw planes (at most the size of the raw payload), owned
 * by the stream and freed with it.
 * Errors: IPC_EINVAL (null argument), IPC_ESTATE (stream of another
 * context), IPC_ENOMEM / IPC_EHIP (device memory or a HIP failure: the stream
 * is left raw and usable).  Returns when the coded form is complete. */
ipc_status ipc_stream_entropy_code(ipc_ctx *ctx, ipc_stream *s);
/* *coding = 0 (raw blocks) or 1 (entropy-coded blocks); IPC_EINVAL on null. */
ipc_status ipc_stream_coding(const ipc_stream *s, int *coding);

/* Per-pass description of a stream (the planner's inputs, Sec. 5). */
typedef struct {
  int32_t level;              /* l (0 for the anchors) */
  int32_t dim;                /* interpolation dimension (-1 for the anchors) */
  uint64_t n_targets;         /* points predicted by the pass */
  uint64_t n_chunks;
  uint64_t plane_bytes[32];   /* stored bytes of plane k over the pass */
  uint32_t errq[33];          /* delta-y in code units with b planes discarded */
  uint32_t progressive;       /* 0 for passes that are always fully loaded */
  uint32_t launch_pass;       /* pass whose timing slot records the kernel launch that
                                 runs this pass (itself unless one launch runs the
                                 whole level; then the level's last pass) */
} ipc_pass_info;

ipc_status ipc_stream_pass_info(const ipc_stream *s, uint32_t pass, ipc_pass_info *out);

/* Alg. 1: reconstruct from the planes the Sec. 5 planner selects for
 * `target`.  The state holds the reconstruction and the plan; `info` may be
 * NULL. */
ipc_status ipc_retrieve(ipc_ctx *ctx, const ipc_stream *s, ipc_target target, ipc_state **out,
                        ipc_info *info);
/* Same, with an explicit plan (planes discarded per pass, n_passes entries). */
ipc_status ipc_retrieve_plan(ipc_ctx *ctx, const ipc_stream *s, const uint8_t *plan,
                             uint32_t n_passes, ipc_state **out, ipc_info *info);
/* Retrieval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reconstruction of ipc_retrieve (same plan, same bytes) written into the
 * caller's `field_dev` (capacity bytes, at least n * itemsize, C order, the
 * stream's dtype), with no state created and no device allocation of any
 * kind.  The fused level path (3-D and 2-D fields with the default chunk
 * shape) keeps its compact coarse grids in a library
 * scratch array of IPC_NOALLOC_SCRATCH_BYTES bytes per device, held from the
 * first context on that device until the process ends; a stream whose coarse
 * grids need more (about n * itemsize / 7, so 3-D fields above roughly
 * 2^25 float32 or 2^24 float64 points) is refused with IPC_EINVAL before any
 * device work.  Other shapes need no scratch.  Every call on a device shares
 * its scratch: calls that overlap on one device (several contexts or host
 * threads) race and must be serialized by the caller.  `info` may be NULL;
 * on an error `field_dev` may be partly written. */
#define IPC_NOALLOC_SCRATCH_BYTES (16u << 20)
ipc_status ipc_retrieve_noalloc(ipc_ctx *ctx, const ipc_stream *s, ipc_target target,
                                void *field_dev, uint64_t capacity, ipc_info *info);
/* Device pointer to the state's reconstructed field x~ of Alg. 1 (C order,
 * the stream's dtype), owned by the state; valid until ipc_state_free, and
 * updated in place by ipc_refine (Alg. 2). */
const void *ipc_state_field(const ipc_state *st);
/* Stream-ordered device-to-device copy of the state's field into `dst_dev`
 * (capacity bytes, at least n * itemsize). */
ipc_status ipc_state_copy_field(ipc_ctx *ctx, const ipc_state *st, void *dst_dev,
                                uint64_t capacity);
/* Number of passes of a stream (anchors + one per level and dimension). */
ipc_status ipc_stream_passes(const ipc_stream *s, uint32_t *n_passes);
/* Alg. 2: tighten a resident reconstruction to `target`, loading only planes
 * not yet loaded; the result equals a fresh retrieval with the new plan bit
 * for bit.  A target already met is a no-op (IPC_FLAG_NOOP). */
ipc_status ipc_refine(ipc_ctx *ctx, ipc_state *st, ipc_target target, ipc_info *info);
void ipc_state_free(ipc_state *st);

/* Refinement in the paper's additive form (Alg. 2, a variant of ipc_refine):
 * plans and reads the new planes as ipc_refine does, then predicts a
 * difference field from itself pass by pass (interpolation is linear) with
 * the code differences of the newly loaded planes, outliers adding nothing,
 * and adds it to the current reconstruction wherever it is not zero.  The
 * result agrees with a fresh retrieval only up to rounding; the reported bound
 * adds a rounding allowance to the plan's bound (the old reconstruction's
 * rounding terms, the difference field's, and u M for the addition).  Runs
 * the one-pass-per-launch kernels for every shape.  Uses a context working
 * buffer of the field's size.  Arguments, no-op cases and errors as for
 * ipc_refine; on an error the state keeps its plan and bound (its field may
 * be partly updated if the failure came from the device). */
ipc_status ipc_refine_additive(ipc_ctx *ctx, ipc_state *st, ipc_target target, ipc_info *info);

/* Batches (beyond the paper, which compresses one field at a time): n fields
 * or streams in one call.  Fields of 3-D or 2-D shape with the default chunk
 * shape share one kernel launch per level (a work list of every field's column
 * segments; a field with fewer levels joins from its top level on), which
 * keeps the device full where single small levels would not.  Results are
 * bit-identical to n separate calls, which is also what other shapes get.
 *
 * ipc_compress_batch: fields_dev[i] with dims[i * ndim ..] and abs_eb[i],
 *   one dtype and one ipc_options for all; out[0..n) receives n streams
 *   (all NULL on error).
 * ipc_retrieve_batch: streams[i] to targets[i]; out[0..n) receives n
 *   states, info (NULL or n entries) their descriptions; t_device_ms is the
 *   batch's device time. */
ipc_status ipc_compress_batch(ipc_ctx *ctx, uint32_t n, const void *const *fields_dev,
                              const uint64_t *dims, int ndim, int dtype, const double *abs_eb,
                              const ipc_options *opts, ipc_stream **out);
ipc_status ipc_retrieve_batch(ipc_ctx *ctx, uint32_t n, const ipc_stream *const *streams,
                              const ipc_target *targets, ipc_state **out, ipc_info *info);

/* One request of a served batch: a retrieval of `stream` (refine = 0; the
 * new state is returned in `state`, which must be NULL on entry) or a
 * refinement of the resident `state` (refine = 1, `stream` ignored), both to
 * `target`.  status and info are outputs. */
typedef struct {
  const ipc_stream *stream;
  ipc_state *state;
  ipc_target target;
  int32_t refine;
  int32_t status;
  ipc_info info;
} ipc_request;

/* A mixed batch of retrievals and refinements (Alg. 1 and Alg. 2 for many
 * requests at once): requests on 3-D streams with the default chunks (of the
 * first such request's dtype and interpolation) share one launch per level,
 * a refinement joining at the level of its first changed pass; the others
 * run one at a time.  Each result equals the same request served alone.
 * Returns IPC_OK when every request was attempted; per-request outcomes are
 * in req[i].status. */
ipc_status ipc_serve_batch(ipc_ctx *ctx, uint32_t n, ipc_request *req);

/* Device bytes of the field a stream reconstructs / a state holds. */
ipc_status ipc_stream_field_bytes(const ipc_stream *s, uint64_t *bytes);
ipc_status ipc_state_field_bytes(const ipc_state *st, uint64_t *bytes);

/* Serving loop (beyond the paper): streams and reconstructions stay
 * resident; requests are submitted from any host thread and served by one
 * worker thread in continuous batches (ipc_serve_batch), admitted in arrival
 * order as their device memory fits `budget_bytes` (a new state's field plus
 * the transient coarse grids; a large request does not hold back smaller
 * ones behind it), at most `max_batch` (0 = 64) per batch.
 *  - ipc_server_submit: a retrieval of `stream` (refine_state NULL) or a
 *    refinement of `refine_state`; IPC_ENOMEM if it can never fit.
 *  - ipc_server_wait: blocks (timeout_ms < 0: no limit; IPC_ESTATE on time
 *    out) until the request is served; returns its status, the state (new
 *    for retrievals, owned by the caller from then on), its info and its
 *    latency from submission to completion.
 *  - ipc_server_release: frees a state the server made (asynchronously; its
 *    memory returns to the budget).
 *  - ipc_server_lock / unlock: exclusive use of the context between batches
 *    (the worker holds it while a batch runs); any other call on the
 *    context while the server exists must be made under it.
 *  - ipc_server_destroy: serves what fits, fails the rest, joins the worker.
 * A refinement and a retrieval of the same state must not be outstanding at
 * once. */
typedef struct ipc_server ipc_server;
ipc_status ipc_server_create(ipc_ctx *ctx, uint64_t budget_bytes, uint32_t max_batch,
                             ipc_server **out);
ipc_status ipc_server_submit(ipc_server *srv, const ipc_stream *stream, ipc_state *refine_state,
                             ipc_target target, uint64_t *ticket);
ipc_status ipc_server_wait(ipc_server *srv, uint64_t ticket, int64_t timeout_ms, ipc_state **state,
                           ipc_info *info, double *latency_ms);
ipc_status ipc_server_release(ipc_server *srv, ipc_state *st);
ipc_status ipc_server_lock(ipc_server *srv);
ipc_status ipc_server_unlock(ipc_server *srv);
ipc_status ipc_server_stats(ipc_server *srv, uint64_t *used, uint64_t *peak, uint64_t *batches,
                            uint64_t *served);
void ipc_server_destroy(ipc_server *srv);

/* Autotuner (beyond the paper): compresses and fully retrieves the given
 * representative field once per candidate column length (chunk rows per
 * workgroup of the fused 3-D level launches: 16, 8, 4, 2, 1; every level at
 * once, twice) and keeps, per level and direction, the fastest launch for
 * this (shape, dtype, interpolation) in the context; later calls on that
 * shape, batched ones included, use the choices.  Outputs never depend on
 * the column length.  zseg_c / zseg_r (NULL, or `capacity` entries indexed
 * by level; 0 = no fused launch) receive the choices.  IPC_EUNSUPPORTED for
 * shapes without fused 3-D launches (2-D fields have one chunk row per
 * column, so nothing to choose).  ipc_autotune_clear forgets every choice. */
ipc_status ipc_autotune(ipc_ctx *ctx, const void *field_dev, const uint64_t *dims, int ndim,
                        int dtype, double abs_eb, const ipc_options *opts, int32_t *zseg_c,
                        int32_t *zseg_r, uint32_t capacity);
ipc_status ipc_autotune_clear(ipc_ctx *ctx);
/* Batch autotuner (beyond the paper): the schedule of batches of `copies`
 * (1..64) copies of a representative field of this (shape, dtype,
 * interpolation), for the automatic batch mode of ipc_ctx_set_batch_graphs.
 * Each candidate is timed three times, in turns, on one compression batch and
 * one full-precision retrieval batch: direct launches, and graph replays whose
 * full queue slots run 3, 4 or 5 (float64: 2, 3 or 4) workgroups per CU for
 * retrieval and 2, 3 or 4 (float64: 1 or 2) for compression.  The choice is
 * kept in the context (ipc_autotune_clear forgets it); `choice` (NULL, or 4
 * entries) receives compression's (graphs 0/1, workgroups per CU), then
 * retrieval's.  Results never depend on the schedule.  IPC_EUNSUPPORTED for
 * shapes without fused launches. */
ipc_status ipc_autotune_batch(ipc_ctx *ctx, const void *field_dev, const uint64_t *dims, int ndim,
                              int dtype, double abs_eb, const ipc_options *opts, uint32_t copies,
                              int32_t choice[4]);
/* Install column lengths chosen earlier (e.g. by ipc_autotune in another
 * process): n entries per direction indexed by level, 0 = default rule. */
ipc_status ipc_autotune_set(ipc_ctx *ctx, const uint64_t *dims, int ndim, int dtype, int interp,
                            const int32_t *zseg_c, const int32_t *zseg_r, uint32_t n);

/* Host-only planner on a serialized stream (no GPU needed): the plan the
 * library would choose for `target`, optionally restricted to b <= limit[s]
 * (refinement).  plan_out has room for the stream's pass count. */
ipc_status ipc_plan_host(const void *stream_bytes, uint64_t nbytes, ipc_target target,
                         const uint8_t *limit, uint8_t *plan_out, uint32_t plan_capacity,
                         double *bound_out, uint32_t *flags_out, uint64_t *loaded_out);

/* Per-pass device timing (for measurement): when on, the pass kernels of
 * later compress / retrieve / refine calls (every pass, or only pass
 * `only_pass` when it is >= 0) are bracketed by HIP events on the context's
 * stream; ipc_ctx_pass_times returns the last call's milliseconds per pass
 * (n_out = the stream's pass count; 0 for passes not timed).  A launch that
 * runs several passes is timed once, in the slot ipc_pass_info.launch_pass
 * names; `only_pass` selects launches by that slot. */
ipc_status ipc_ctx_set_profiling(ipc_ctx *ctx, int on, int only_pass);
ipc_status ipc_ctx_pass_times(const ipc_ctx *ctx, float *ms, uint32_t capacity, uint32_t *n_out);

/* Batched retrievals as graph replays (the batching of many uneven fields by
 * one persistent launch per level that the problem statement asks for).
 * When on, ipc_retrieve_batch and the retrievals and refinements of
 * ipc_serve_batch over fused streams (3-D and 2-D fields with the default
 * chunk shape; at most 2048 of them and 16384 level work lists per call) run as
 * queue launches: the per-field head jobs, then for each level one
 * persistent grid whose workgroups claim column segments of every field at
 * that level from a device counter.  Everything that varies from batch to
 * batch is uploaded as one table, so the launch sequence is captured once
 * per launch shape (dtype, interpolation, number of levels, grid class of
 * each level) into a HIP graph and replayed after.  Results are identical to
 * the direct launches (the same kernels' bodies).  Graphs, the device table
 * (about 10 MB) and its pinned staging copy live until ipc_ctx_destroy.
 * `on`: 0 = direct launches (the default), 2 = automatic (the schedule
 * ipc_autotune_batch chose when every field of the batch has that tuned
 * shape, else graph replays only when no field exceeds 2^22 points: on large
 * fields the launch overhead a replay saves is small against the work), any
 * other value = always graph replays (the Python Server's setting: serving
 * mixes ran 22-26 % more requests per second with it).  Compression batches
 * follow the same setting.  If the context's stream cannot be captured, the
 * call runs the direct launches and the setting turns itself off.
 * ipc_ctx_graph_stats counts captured graphs and replays. */
ipc_status ipc_ctx_set_batch_graphs(ipc_ctx *ctx, int on);
ipc_status ipc_ctx_graph_stats(const ipc_ctx *ctx, uint64_t *captured, uint64_t *replays);

const char *ipc_status_string(ipc_status st);
const char *ipc_last_error(const ipc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* IPCOMP_H */
