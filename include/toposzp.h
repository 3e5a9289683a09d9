/*
 * toposzp.h -- C ABI of the MI355X (gfx950) TopoSZp library, libtoposzp.so.
 *
 * TopoSZp (topology-aware SZp) compresses a float32 scalar field on a
 * structured grid into a byte stream whose reconstruction keeps every point
 * within a relaxed but enforced bound (|a - a^| <= 2e) and never introduces a
 * new critical point or changes a critical point's type, while restoring the
 * minima, maxima and saddles that plain error-bounded quantization flattens
 * (problem statement: Section III; pipeline: Section IV).
 *
 * Conventions for every call below:
 *  - Pointers named d_* are DEVICE pointers (HIP global memory on the
 *    current device); h_* are host pointers.  The caller owns every buffer;
 *    the library never allocates, frees or retains memory (one exception:
 *    the scratch of toposzp_compress_noalloc).  Alignment: the
 *    input field 16 bytes, streams and sizes 8 bytes, the workspace 256
 *    bytes, reconstructions and statuses 4 bytes (TOPOSZP_E_INVALID_ARG
 *    otherwise).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are stream-ordered and asynchronous: results are valid once the
 *    stream has been synchronised.  Nothing is read back to the host except
 *    where a call says so (the stats calls, the autotuners).
 *  - The return value is a status: TOPOSZP_OK (0) or a negative error from
 *    the list below, detected on the host before anything is enqueued.
 *    Errors that only the device can see (non-finite input, values out of
 *    quantizer range, a corrupt stream) are written to *d_status (int32,
 *    device) when the enqueued work completes; *d_status is always written.
 *  - Grid dimensions are in C order, slowest first: 2D = {ny, nx},
 *    3D = {nz, ny, nx}; x varies fastest.  A field holds at most 2^31 - 1
 *    points.
 *  - One workspace serves one call at a time: calls that share a workspace
 *    must be ordered on one stream.  Calls on different workspaces may be
 *    issued from several host threads at once.
 *  - No exception crosses the ABI.
 */
#ifndef TOPOSZP_H
#define TOPOSZP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TOPOSZP_OK 0
#define TOPOSZP_E_INVALID_ARG (-1) /* bad ndim, dims, bound, params, pointer */
#define TOPOSZP_E_NONFINITE (-2)   /* NaN or Inf in the input field */
#define TOPOSZP_E_RANGE (-3)       /* bound below 2^-100 or above 2^100 (after
                                      rounding down to float), or some |q|
                                      would exceed 2^22 - 1 */
#define TOPOSZP_E_CAPACITY (-4)    /* output or workspace too small */
#define TOPOSZP_E_CORRUPT (-5)     /* stream fails a header/segment check */
#define TOPOSZP_E_DEVICE (-6)      /* a HIP runtime call failed */
#define TOPOSZP_E_UNSUPPORTED (-7) /* valid request this build cannot run */

#define TOPOSZP_EB_ABS 0 /* e = eb */
#define TOPOSZP_EB_REL 1 /* e = eb * (max - min) of the field (eb if flat) */

/* Compression parameters; pass NULL for the defaults shown. */
typedef struct {
  uint32_t block;     /* points per block; must be 64 (default 64) */
  int32_t rank_scope; /* 0 = ranks among flattened extrema of the same 64-point
                         block (default); 1 = whole field (needs the _ex sizes;
                         the flattened extrema are sorted on the device, with
                         every count kept there, so the call is as
                         asynchronous as the block-scope one; not in the
                         batched form: TOPOSZP_E_UNSUPPORTED there) */
  int32_t rbf_policy; /* 0 = adaptive kernel size/width (default),
                         1 = always k_size 3 */
  int32_t max_rounds; /* cap on saddle-refinement rounds, 1..65535 (16) */
  int32_t topo;       /* 1 = TopoSZp (default), 0 = plain SZp stream */
} toposzp_params;

/* Header fields of a stream, as parsed on the host by toposzp_inspect. */
typedef struct {
  int32_t ndim, topo, rank_scope, eb_mode, k_size, max_rounds;
  uint64_t dims[3]; /* C order; unused trailing entries are 1 */
  uint64_t n, nblocks, total_bytes, data_planes, rank_planes;
  double eb, eps;   /* requested bound and the absolute bound it implies */
  float e;          /* the float32 bound the quantizer used */
  float vmin, vmax; /* field range (relative mode; 0 in absolute mode) */
  float sigma;      /* Gaussian width of the saddle refinement */
} toposzp_info;

/* Stream format version written by this library (1). */
int toposzp_version(void);

/* Static message for a status code. */
const char *toposzp_strerror(int status);

/* Worst-case stream size in bytes for a field of these dims (header, the
 * fixed-size parts and payloads at their maximum widths).  0 if the dims are
 * invalid.  `dims` is a host array of `ndim` entries. */
size_t toposzp_compress_bound(uint32_t ndim, const uint64_t *dims);

/* Device workspace bytes that compression and decompression of a field of
 * these dims need (one size serves both).  0 if the dims are invalid. */
size_t toposzp_workspace_size(uint32_t ndim, const uint64_t *dims);

/* The same two sizes for a rank scope (params.rank_scope: 0 block, 1 field).
 * Field-scope ranks reach 31 bits, and their compression sorts the
 * flattened extrema of the whole field, so both sizes are larger. */
size_t toposzp_compress_bound_ex(uint32_t ndim, const uint64_t *dims, int32_t rank_scope);
size_t toposzp_workspace_size_ex(uint32_t ndim, const uint64_t *dims, int32_t rank_scope);

/* Clears a freshly allocated workspace (enqueued on `stream`).  Must be called
 * once before a workspace's first use and again after any call on it that
 * failed with TOPOSZP_E_DEVICE; every successful call leaves it reusable. */
int toposzp_workspace_init(void *d_ws, size_t ws_bytes, void *stream);

/* Compression (Section IV-A): critical point detection and ranks on the
 * original values, quantization to bin indices, per-64-point blocking with
 * 1-D difference decorrelation, fixed-length bit-plane encoding, and the
 * same blocking/encoding applied again to the rank metadata.
 *   d_field    : N float32 values, C order, device.
 *   eb_mode/eb : TOPOSZP_EB_ABS or TOPOSZP_EB_REL; eb > 0 and finite.
 *   d_out      : device byte buffer of out_cap bytes; out_cap must be at least
 *                toposzp_compress_bound(ndim, dims).
 *   d_out_size : device uint64, receives the stream length (0 on error).
 *   d_status   : device int32, receives TOPOSZP_OK or a device-side error.
 * The stream layout is described in the project's design notes (header,
 * fixed-size parts, then the two bit-plane payloads). */
int toposzp_compress(const float *d_field, uint32_t ndim, const uint64_t *dims,
                     int eb_mode, double eb, const toposzp_params *params,
                     void *d_ws, size_t ws_bytes, uint8_t *d_out,
                     size_t out_cap, uint64_t *d_out_size, int32_t *d_status,
                     void *stream);

/* Allocation-free compression, for callers that cannot allocate device memory
 * (work under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): toposzp_compress with block-scope ranks, minus the workspace.
 * Its kernels use a scratch array inside the library instead, one per device
 * (62,985,216 bytes, held from the library's load until the process ends);
 * the call itself allocates and frees nothing.  The caller still owns the
 * field, the output, the size and the status, with the meanings and
 * alignments of toposzp_compress.
 *  - Fields of at most TOPOSZP_NOALLOC_MAX_POINTS (2^24) points; larger ones
 *    return TOPOSZP_E_CAPACITY before anything is enqueued.
 *  - params.rank_scope 1 (field scope) returns TOPOSZP_E_UNSUPPORTED.
 *  - Every call on a device shares that device's scratch, which keeps the last
 *    call's contents (no call depends on them).  Calls on one device must be
 *    ordered (one stream, or synchronised): calls that overlap race and give
 *    undefined streams.
 * The stream equals toposzp_compress's for the same arguments. */
#define TOPOSZP_NOALLOC_MAX_POINTS (1ull << 24)
int toposzp_compress_noalloc(const float *d_field, uint32_t ndim, const uint64_t *dims,
                             int eb_mode, double eb, const toposzp_params *params,
                             uint8_t *d_out, size_t out_cap, uint64_t *d_out_size,
                             int32_t *d_status, void *stream);

/* Decompression (Section IV-B): decoding to bin-centre values, metadata
 * extraction, the extrema stencil on flattened minima/maxima and iterated
 * RBF refinement of flattened saddles with the guard against new or changed
 * critical points.
 *   d_in/in_size : device stream and its length in bytes.
 *   d_out        : device float32 buffer of out_cap_elems values; receives the
 *                  N-point reconstruction in C order (N from the stream; the
 *                  call fails with TOPOSZP_E_CAPACITY status if N exceeds
 *                  out_cap_elems).
 *   d_status     : device int32, receives TOPOSZP_OK, TOPOSZP_E_CORRUPT or
 *                  TOPOSZP_E_CAPACITY.
 * The workspace must have been sized for at least the stream's dims. */
int toposzp_decompress(const uint8_t *d_in, size_t in_size, float *d_out,
                       size_t out_cap_elems, void *d_ws, size_t ws_bytes,
                       int32_t *d_status, void *stream);

/* Blocking conveniences: enqueue, synchronise `stream`, and return the
 * device status (or the host error).  *h_out_size receives the stream length
 * (compress). */
int toposzp_compress_sync(const float *d_field, uint32_t ndim,
                          const uint64_t *dims, int eb_mode, double eb,
                          const toposzp_params *params, void *d_ws,
                          size_t ws_bytes, uint8_t *d_out, size_t out_cap,
                          uint64_t *h_out_size, void *stream);
int toposzp_decompress_sync(const uint8_t *d_in, size_t in_size, float *d_out,
                            size_t out_cap_elems, void *d_ws, size_t ws_bytes,
                            void *stream);

/* Topological errors of a reconstruction against its original (Section
 * III-B), computed on the device with the library's classifier.  d_orig and
 * d_recon: N float32 values each (dims as for compression).  d_counts
 * (int64[11], device) receives FN, FP, FT, then the original's points by class
 * r, m, s, M, then FN by original class r, m, s, M; d_max_err (double,
 * device) the largest |orig - recon|.  Both are overwritten. */
int toposzp_eval(const float *d_orig, const float *d_recon, uint32_t ndim, const uint64_t *dims,
                 int64_t *d_counts, double *d_max_err, void *stream);

/* ---- Batched form: many fields of uneven sizes per call (one launch per
 * stage for the whole batch; every field's stream and reconstruction are
 * those of a one-field call).  Job arrays are host arrays of `count`
 * entries (1..4096), read during the call only; every pointer inside a job
 * is a device pointer with the alignment of the one-field calls.  The
 * workspace (sized by the *_workspace_size calls, cleared once with
 * toposzp_workspace_init) holds a job table and one workspace per job; a
 * batch call copies the table into it on `stream`.  Host-detected errors in
 * any job fail the whole call before anything is enqueued; device-side
 * results and errors go to each job's own size/status. */
typedef struct {
  const float *d_field; /* N float32 values, C order */
  uint32_t ndim;        /* 2 or 3 */
  uint64_t dims[3];     /* C order; unused entries ignored */
  int32_t eb_mode;      /* TOPOSZP_EB_ABS or TOPOSZP_EB_REL */
  double eb;
  uint8_t *d_out;       /* out_cap >= toposzp_compress_bound(ndim, dims) */
  size_t out_cap;
  uint64_t *d_out_size; /* device uint64: stream length */
  int32_t *d_status;    /* device int32: status of this job */
} toposzp_compress_job;

typedef struct {
  const uint8_t *d_in; /* stream */
  size_t in_size;
  float *d_out;        /* reconstruction, out_cap_elems values */
  size_t out_cap_elems;
  int32_t *d_status;   /* device int32: status of this job */
} toposzp_decompress_job;

size_t toposzp_compress_batch_workspace_size(uint32_t count, const toposzp_compress_job *h_jobs);
size_t toposzp_decompress_batch_workspace_size(uint32_t count, const toposzp_decompress_job *h_jobs);
int toposzp_compress_batch(uint32_t count, const toposzp_compress_job *h_jobs, const toposzp_params *params,
                           void *d_ws, size_t ws_bytes, void *stream);
int toposzp_decompress_batch(uint32_t count, const toposzp_decompress_job *h_jobs, void *d_ws, size_t ws_bytes,
                             void *stream);
/* Counters (as toposzp_decompress_stats, with the same conditions) of job
 * `index` of the last batched decompression on this workspace with these
 * jobs. */
int toposzp_decompress_batch_stats(uint32_t count, const toposzp_decompress_job *h_jobs, void *d_ws,
                                   uint32_t index, int64_t out[5], void *stream);

/* Launch shapes used by every call of this process (they change no byte of
 * any result): waves per workgroup of the encode and decode kernels (4 or 8)
 * and the persistent grid of the batched form in workgroups per compute
 * unit (1..32).  Defaults {8, 4, 8, 8}.  Calls on other host threads read
 * either the old or the new set, never a mix. */
typedef struct {
  int32_t encode_waves, decode_waves, compress_wgs_per_cu, decompress_wgs_per_cu;
} toposzp_tuning;
int toposzp_set_tuning(const toposzp_tuning *t);
int toposzp_get_tuning(toposzp_tuning *t);
/* Autotuner: runs the given batch under each candidate shape (encode or
 * decode waves x workgroups per CU), times it with HIP events on `stream`
 * (synchronising it), keeps the fastest as the current tuning and returns it
 * in *out.  The batch's outputs are written as by an ordinary call. */
int toposzp_autotune_compress_batch(uint32_t count, const toposzp_compress_job *h_jobs,
                                    const toposzp_params *params, void *d_ws, size_t ws_bytes, void *stream,
                                    toposzp_tuning *out);
int toposzp_autotune_decompress_batch(uint32_t count, const toposzp_decompress_job *h_jobs, void *d_ws,
                                      size_t ws_bytes, void *stream, toposzp_tuning *out);

/* Parses and checks a stream header held in host memory (at least 512
 * bytes, the header of d_in copied to the host).  Returns TOPOSZP_OK or
 * TOPOSZP_E_CORRUPT. */
int toposzp_inspect(const uint8_t *h_hdr, size_t n, toposzp_info *out);

/* Counters of the last decompression on this workspace: out[0] refinement
 * rounds run, [1] saddle updates committed, [2] flattened saddles queued,
 * [3] extrema moved by the stencil, [4] flattened extrema left in place by
 * the error budget.  They are gathered on request from what the
 * decompression left in the workspace: call this on the decompression's
 * stream before any other call uses the workspace.  Enqueues one small
 * kernel that writes the control block of d_ws, then synchronises `stream`. */
int toposzp_decompress_stats(void *d_ws, int64_t out[5], void *stream);

/* Per-kernel timing with HIP events on the call's stream (a diagnostic for
 * one host thread and one device: the events are shared by all calls).
 * While enabled, each call records events around its kernels; after the
 * stream is synchronised toposzp_kernel_times fills ms[] for the last
 * compress and decompress: [0] range pass, [1] encode, [2] finalize,
 * [3] decode, [4] refine; -1 where a kernel did not run.  Returns the count
 * written. */
int toposzp_set_timing(int enable);
int toposzp_kernel_times(float *ms, int max);

#ifdef __cplusplus
}
#endif
#endif /* TOPOSZP_H */
