/*
 * aolmi.h -- Array-OL repetitive tasks on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the downscaler hot path from Rodrigues, Guyomarc'h, Dekeyser,
 * "Programming Massively Parallel Architectures using MARTE: a Case Study":
 * a video downscaler written as Array-OL repetitive tasks (Sec. III-A), i.e.
 * tilers that take each pattern at origin + paving.r + fitting.i modulo the
 * array shape, and an elementary per-pattern filter: a horizontal then a
 * vertical polyphase interpolating filter over every frame and colour plane
 * (Sec. III).
 *
 * General rules
 *  - Every function returns an aol_status. Functions never throw, abort or
 *    print; on failure aol_last_error() returns a thread-local message.
 *  - Device buffers are plain device pointers owned by the caller. Plans own
 *    the device tables they allocate at creation (filter fragments, tile
 *    lists, pointer tables) and free them on destroy.
 *  - Run calls (aol_downscale_u8, aol_downscale_f, aol_downscale_u8_unfused,
 *    aol_downscale_u8_unfused_static, aol_batch_run, aol_batch_run_buffers,
 *    aol_graph_launch, aol_wsum_run, aol_linear_run) only enqueue work on the given stream:
 *    they never allocate and never synchronise. They check pointers and
 *    alignment and report launch errors; faults inside a kernel surface at
 *    the caller's next synchronisation.
 *  - Inputs and outputs must not alias.
 *  - Distinct plans may be used from different threads; one plan is not
 *    re-entrant (do not run it on two streams at once).
 *  - Streams are hipStream_t; NULL is the default stream.
 */
#ifndef AOLMI_H
#define AOLMI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum aol_status {
  AOL_OK = 0,
  AOL_ERR_INVALID = -1,     /* bad shape, rank, pointer, pitch or argument */
  AOL_ERR_UNSUPPORTED = -2, /* legal request outside the implemented limits */
  AOL_ERR_NOMEM = -3,       /* host or device allocation failed */
  AOL_ERR_HIP = -4          /* a HIP runtime call failed (see aol_last_error) */
} aol_status;

typedef enum aol_precision {
  AOL_PREC_U8 = 0,   /* uint8 pixels, integer taps, bit-exact fixed point */
  AOL_PREC_BF16 = 1, /* bfloat16 normalised pixels in, float32 out (MFMA) */
  AOL_PREC_FP16 = 2  /* float16 normalised pixels in, float32 out (MFMA) */
} aol_precision;

/* Implementation limits (AOL_ERR_UNSUPPORTED beyond these). */
#define AOL_MAX_P 16        /* output phases per repetition */
#define AOL_MAX_Q 64        /* input pixels per repetition */
#define AOL_MAX_TAPS 32     /* taps per phase */
#define AOL_MAX_COEFF 2047  /* |c| for integer taps */
#define AOL_MAX_PLANES 4    /* planes per downscale plan */
#define AOL_MAX_RANK 4      /* ranks of generic tilers */

/* Thread-local text of the last error (never NULL; empty after success). */
const char* aol_last_error(void);

/* Library version, "major.minor.patch". */
const char* aol_version(void);

/* --------------------------------------------------------------------------
 * One axis of the downscaler: a polyphase interpolating filter.
 *
 * Sec. III: the horizontal filter reduces each line (352 -> 132 pixels in the
 * paper's CIF case) and the vertical filter reduces the lines (288 -> 128),
 * each by interpolating packets of input pixels. Sec. III-A: the horizontal
 * task has multiplicity [288, 44], one elementary task per line and packet.
 * Here a repetition r consumes a packet of q input pixels and emits p output
 * pixels; on an axis of length N there are R = ceil(N/q) repetitions and
 * M = p*R outputs. Output o = p*r + phi (phase phi < p) is
 *
 *   acc = sum_{k<taps} coeff[phi*taps + k] * x[(q*r + s_phi + k) mod N]
 *
 * integer path: out = clamp(floor((acc + 128) / 256), 0, 255);
 * float path:   out = acc / 256 evaluated in float (no clamp).
 *
 * The paper gives no coefficients, tap count or window placement; they are
 * caller data. phase_start (host, p entries) gives s_phi; NULL selects the
 * pixel-centre default s_phi = floor(((2phi+1)q - p) / (2p)) - floor((taps-1)/2),
 * see aol_default_phase_starts. coeff is host memory, p*taps int16, row-major
 * [phase][tap]; it is copied at plan creation.
 * ------------------------------------------------------------------------ */
typedef struct aol_polyphase {
  int32_t p;
  int32_t q;
  int32_t taps;
  const int16_t* coeff;       /* host, [p][taps] */
  const int32_t* phase_start; /* host, [p], or NULL for the default */
} aol_polyphase;

/* Default window starts for (p, q, taps) into out[0..p). AOL_ERR_INVALID if
 * any argument is < 1 or out is NULL. */
aol_status aol_default_phase_starts(int32_t p, int32_t q, int32_t taps, int32_t* out);

/* Output size of a h x w plane: out_h = vf.p*ceil(h/vf.q), out_w =
 * hf.p*ceil(w/hf.q). The only way callers learn output sizes. */
aol_status aol_downscale_output_shape(int64_t h, int64_t w, const aol_polyphase* hf,
                                      const aol_polyphase* vf, int64_t* out_h, int64_t* out_w);

/* --------------------------------------------------------------------------
 * Frame downscaler plans (Sec. III: horizontal filter then vertical filter,
 * repeated for every frame and every colour plane; the two filters are fused
 * in one kernel and the intermediate frame never leaves the chip).
 *
 * One plan covers up to AOL_MAX_PLANES planes (e.g. Y, U, V of I420), all
 * filtered with the same hf (along each line) and vf (along each column).
 * Pitches are in elements of the plane's type (uint8 for AOL_PREC_U8; 16-bit
 * for the float input; float32 for the float output); 0 means tightly
 * packed. The integer path rounds the intermediate to uint8 after the
 * horizontal pass, exactly as two separate filters exchanging a uint8 frame.
 * ------------------------------------------------------------------------ */
typedef struct aol_plane_desc {
  int64_t height;
  int64_t width;
  int64_t in_pitch;  /* elements between input rows, >= width, or 0 */
  int64_t out_pitch; /* elements between output rows, >= output width, or 0 */
} aol_plane_desc;

typedef struct aol_plan aol_plan;

/* Validate shapes and filters, build the device tables. AOL_ERR_UNSUPPORTED
 * for p > AOL_MAX_P, q > AOL_MAX_Q, taps > AOL_MAX_TAPS, |coeff| >
 * AOL_MAX_COEFF (U8), coefficients whose c/256 is not exact in the chosen
 * float format (BF16: at most 8 significant bits), or planes whose height or
 * width exceeds 2^30. */
aol_status aol_downscale_plan_create(const aol_plane_desc* planes, int32_t n_planes,
                                     const aol_polyphase* hf, const aol_polyphase* vf,
                                     aol_precision prec, aol_plan** out);
aol_status aol_plan_destroy(aol_plan* plan);

/* Tiled schedule: selects the 2-D tile kernel (input tile with halo and the
 * intermediate tile in LDS) with this tile shape in repetitions (tile_rx along
 * lines, tile_ry along columns). tile_rx*hf.q must be a multiple of 16 elements (U8) or 8
 * (float); at most 512 outputs per tile and axis. AOL_ERR_INVALID for a
 * misaligned tile, AOL_ERR_UNSUPPORTED if it would not fit the chip's shared
 * memory. Optional: plans start with about 128 input pixels per tile side.
 * Rebuilds the plan's tables like aol_plan_set_band (capture graphs again). */
aol_status aol_plan_set_tile(aol_plan* plan, int32_t tile_rx, int32_t tile_ry);

/* Band schedule (the default for every plan that fits it): a workgroup owns a
 * column band of band_reps repetitions (0: the widest that fits a compute
 * unit, normally the full width) and streams segments of seg_reps
 * repetitions down the plane, keeping the intermediate in an LDS ring.
 * seg_reps 0: the plan keeps unit lists for segments of about 512, 256, 128
 * and 64 input lines, and each launch takes the longest that leaves every
 * resident workgroup about four units. Multiples of 16. This call (like plan
 * creation) builds and uploads those lists synchronously; it frees the
 * previous ones, so a graph captured from an earlier run of this plan must
 * be captured again. Selecting a band re-selects the band kernel after
 * aol_plan_set_tile. AOL_ERR_UNSUPPORTED if the band does not fit. Results
 * are identical for every schedule. */
aol_status aol_plan_set_band(aol_plan* plan, int32_t band_reps, int32_t seg_reps);

/* Order in which each workgroup walks its contiguous run of tiles inside a
 * plane: 0 = row-major (horizontal neighbours consecutive, the default),
 * 1 = column-major. A schedule choice only; results are identical. */
aol_status aol_plan_set_walk(aol_plan* plan, int32_t order);

/* The schedule a launch of n_frames frames uses, as a JSON object (kernel,
 * segment length, units per frame, items, grid, LDS bytes); plan-owned text,
 * valid until the next call on the plan. "" for a NULL plan. */
const char* aol_plan_schedule(aol_plan* plan, int32_t n_frames);

/* Integer path (plan precision AOL_PREC_U8). For plane j, d_in[j] points to
 * frame 0 of n_frames frames spaced in_frame_stride[j] elements apart, and
 * d_out[j] to the outputs spaced out_frame_stride[j] apart. Host arrays of
 * length n_planes. Vector loads need 16-byte aligned rows and 4-byte aligned
 * output rows; other layouts take a slower element-wise path. */
aol_status aol_downscale_u8(aol_plan* plan, int32_t n_frames, const uint8_t* const* d_in,
                            const int64_t* in_frame_stride, uint8_t* const* d_out,
                            const int64_t* out_frame_stride, hipStream_t stream);

/* Float path (AOL_PREC_BF16 / AOL_PREC_FP16): inputs are 16-bit bit patterns
 * of normalised pixels, outputs float32, weights coeff/256 applied on the
 * matrix cores with float32 accumulation; the intermediate is kept on chip
 * as a hi/lo pair of 16-bit values. */
aol_status aol_downscale_f(aol_plan* plan, int32_t n_frames, const void* const* d_in,
                           const int64_t* in_frame_stride, float* const* d_out,
                           const int64_t* out_frame_stride, hipStream_t stream);

/* --------------------------------------------------------------------------
 * Unfused form of an integer plan (Sec. III-A: the horizontal and the
 * vertical filter are separate repetitive tasks connected by the
 * intermediate frame array). Two kernels per group of frames: the first
 * filters every line and writes the uint8 intermediate, transposed, into a
 * caller-supplied device workspace; the second filters every row of that
 * (i.e. every column of the intermediate) and writes the outputs. Results
 * are identical to aol_downscale_u8, bit for bit; the intermediate makes one
 * round trip through memory, which the fused kernel avoids.
 * ------------------------------------------------------------------------ */

/* Workspace bytes one frame of the plan's planes needs (its transposed
 * intermediates, rows padded to 128 bytes). AOL_ERR_INVALID for a float
 * plan, AOL_ERR_UNSUPPORTED for filters whose 16-output blocks span more
 * than four K-steps of 64 pixels. */
aol_status aol_unfused_workspace_bytes(aol_plan* plan, int64_t* bytes_per_frame);

/* Arguments as aol_downscale_u8, plus d_work: device memory of work_bytes
 * bytes, 256-byte aligned, owned by the caller, not aliasing any input or
 * output. Frames run in groups of floor(work_bytes / bytes_per_frame), in
 * order, on stream (AOL_ERR_INVALID if the workspace holds no frame). The
 * workspace's contents are scratch: the caller must not use it while the
 * call's work is in flight. Enqueue only; vector loads need 16-byte aligned
 * input rows, other layouts take a byte-wise path. */
aol_status aol_downscale_u8_unfused(aol_plan* plan, int32_t n_frames, const uint8_t* const* d_in,
                                    const int64_t* in_frame_stride, uint8_t* const* d_out,
                                    const int64_t* out_frame_stride, void* d_work, int64_t work_bytes,
                                    hipStream_t stream);

/* The same two passes with the intermediate in a static device workspace
 * of 64 MiB (one per GPU, held until the process ends) instead of a
 * caller's: for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid allocation). The call
 * allocates nothing. Frames run in groups that fit the 64 MiB;
 * AOL_ERR_UNSUPPORTED when one frame's intermediate
 * (aol_unfused_workspace_bytes) exceeds it. Every call on a GPU shares that
 * GPU's workspace and nothing in it needs to start cleared: calls that
 * overlap on one GPU (other streams, other threads, other plans) race and
 * must be ordered by the caller. */
aol_status aol_downscale_u8_unfused_static(aol_plan* plan, int32_t n_frames, const uint8_t* const* d_in,
                                           const int64_t* in_frame_stride, uint8_t* const* d_out,
                                           const int64_t* out_frame_stride, hipStream_t stream);

/* --------------------------------------------------------------------------
 * Host-to-host frame pipeline (Sec. IV: in the paper's measurements the
 * copies between host and device memory take most of the application's
 * time, and its tuning removes redundant ones). Frames live in host memory;
 * groups of batch_frames frames are copied to the device on one stream,
 * downscaled by the plan's fused kernel on the caller's stream and copied
 * back on another stream, with `depth` groups in flight in a ring of device
 * slots, so the copies of one group overlap the kernel of another. Host
 * buffers should be pinned (hipHostMalloc, or torch's pin_memory=True) for
 * the copies to run asynchronously; pageable memory works but its copies
 * are staged by the runtime.
 * ------------------------------------------------------------------------ */
typedef struct aol_pipeline aol_pipeline;

typedef struct aol_pipeline_stats {
  int32_t groups;     /* groups of frames moved */
  int32_t frames;
  double wall_ms;     /* host time of the call */
  double span_ms;     /* first host-to-device copy start to last device-to-host copy end (GPU clock) */
  double h2d_ms;      /* sums over the groups of each stage's duration (GPU clock) */
  double kernel_ms;
  double d2h_ms;
  int64_t h2d_bytes;  /* bytes copied each way */
  int64_t d2h_bytes;
} aol_pipeline_stats;

/* Allocates the device slots (depth x batch_frames frames of every plane of
 * an integer plan, in and out) and two copy streams of the default
 * priority. The plan must outlive the pipeline. AOL_ERR_INVALID for a float
 * plan, batch_frames < 1 or depth outside 1..64. */
aol_status aol_pipeline_create(aol_plan* plan, int32_t batch_frames, int32_t depth, aol_pipeline** out);
aol_status aol_pipeline_destroy(aol_pipeline* pipe);

/* h_in[j] / h_out[j]: host memory of frame 0 of plane j, frames
 * in_frame_stride[j] / out_frame_stride[j] bytes apart, rows at the plan's
 * pitches. Outputs are bit-identical to aol_downscale_u8. Not a run call: it
 * enqueues the three stages group by group, waits on the host before reusing
 * a slot, and returns once every output is in host memory. stats may be
 * NULL. One call at a time per pipeline. With n_frames 0 the buffers are not
 * read and may be NULL. */
aol_status aol_pipeline_run_u8(aol_pipeline* pipe, int32_t n_frames, const uint8_t* const* h_in,
                               const int64_t* in_frame_stride, uint8_t* const* h_out,
                               const int64_t* out_frame_stride, hipStream_t stream, aol_pipeline_stats* stats);

/* --------------------------------------------------------------------------
 * Batches of video streams (Sec. III: the downscaler repeats for every frame;
 * Sec. III-A: all elementary tasks are independent, so frames of different
 * streams may run together). One step downscales one frame of every stream,
 * each with its own size and filter pair, in one persistent launch.
 *
 * Device pointers live in a plan-owned device table written by
 * aol_batch_set_pointers (a small enqueued kernel: no host synchronisation),
 * so aol_batch_run -- or a graph captured from it -- is the same launch every
 * step. Batch buffers must be 16-byte aligned; pitches are in elements. Call
 * order per step: aol_batch_set_pointers, then aol_batch_run or
 * aol_graph_launch, on the same stream.
 * ------------------------------------------------------------------------ */
typedef struct aol_stream_desc {
  int64_t height;
  int64_t width;
  int64_t in_pitch;  /* elements, or 0 */
  int64_t out_pitch; /* elements, or 0 */
  aol_polyphase hf;  /* along lines (copied at plan creation) */
  aol_polyphase vf;  /* along columns */
} aol_stream_desc;

typedef struct aol_batch_plan aol_batch_plan;
typedef struct aol_graph aol_graph;
typedef struct aol_buffer_set aol_buffer_set;

/* tune_cache: path of a text file of tuned schedules (read here, appended
 * by aol_autotune), or NULL. All streams use precision prec. */
aol_status aol_batch_plan_create(int32_t n_streams, const aol_stream_desc* streams, aol_precision prec,
                                 const char* tune_cache, aol_batch_plan** out);
aol_status aol_batch_plan_destroy(aol_batch_plan* plan);

/* d_in[i] / d_out[i]: the current frame of stream i (host arrays of device
 * pointers, length n_streams). Enqueued on stream. */
aol_status aol_batch_set_pointers(aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                  hipStream_t stream);

/* One step: every stream's frame at the pointers last set. */
aol_status aol_batch_run(aol_batch_plan* plan, hipStream_t stream);

/* Capture one aol_batch_run into a graph (stream must not be the default
 * stream). Graphs read the pointer table at run time. aol_autotune changes
 * the launch: aol_graph_launch returns AOL_ERR_INVALID for a graph captured
 * before it (capture again), and for a graph whose plan was destroyed. */
aol_status aol_batch_graph_create(aol_batch_plan* plan, hipStream_t stream, aol_graph** out);

/* Capture one step on a fixed buffer set (d_in[i] / d_out[i], checked as by
 * aol_batch_set_pointers) into a graph that holds its own pointer table
 * (allocated and filled here; the plan's table is not touched): a serving
 * loop over a ring of frame slots keeps one graph per slot and launches one
 * graph, one kernel, per step. The buffers must stay valid while the graph
 * is used. The same rules as aol_batch_graph_create apply (non-default
 * stream; invalid after aol_autotune or the plan's destruction). */
aol_status aol_batch_graph_create_pointers(aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                           hipStream_t stream, aol_graph** out);
aol_status aol_graph_launch(aol_graph* graph, hipStream_t stream);
aol_status aol_graph_destroy(aol_graph* graph);

/* A buffer set: one frame's buffers of every stream (d_in, d_out: n device
 * pointers each, 16-byte aligned, checked here) in a pointer table of its own,
 * uploaded now (a configuration call: allocates and synchronises). A serving
 * loop over a ring of frame buffers makes one set per slot and runs each step
 * with aol_batch_run_buffers: one launch, no pointer update. A set belongs to
 * the plan it was made for and stays valid across that plan's schedule
 * changes (aol_autotune, aol_batch_set_schedule); it holds no reference to the
 * buffers, which the caller keeps alive. Destroy sets before or after their
 * plan, in any order. */
aol_status aol_batch_buffers_create(aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                    aol_buffer_set** out);
/* Run call: the plan's launch over the set's buffers (the plan's own pointer
 * table is neither read nor changed). Launches over different sets share only
 * read-only tables, so they may run concurrently on different streams (a
 * serving loop alternating two streams overlaps one step's last workgroups
 * with the next step's first). AOL_ERR_INVALID for a set made for another
 * plan. */
aol_status aol_batch_run_buffers(aol_batch_plan* plan, const aol_buffer_set* set, hipStream_t stream);
aol_status aol_batch_buffers_destroy(aol_buffer_set* set);

/* Times schedule candidates on the buffers last set: first one segment
 * length for every stream x the column-band LDS budget (16..128 repetitions x
 * 150 or 76 KiB); then, where the int8-tap and split-tap streams share one
 * launch, the weight of the int8-tap part in the division of the workgroups
 * (500..1500 per mille); then, classes with the most input first, each stream
 * class's own segment length (16..128; a class: the two ratios and the width
 * class up to 640, 1280, 1920 pixels or wider) with the others held; last the
 * weight again within 100 per mille of the best. Keeps the fastest and appends
 * it to the tuning cache (keyed by the device architecture, the precision and
 * the streams' sizes and filters). Synchronises the stream (not a run call);
 * results are unchanged. */
aol_status aol_autotune(aol_batch_plan* plan, hipStream_t stream);

/* Rebuilds the plan with one schedule: segments of seg_reps repetitions (a
 * multiple of 16; 0: about 512 input lines, shortened for streams whose units
 * would exceed a workgroup's fair share) and column bands that fit
 * lds_budget bytes of LDS per workgroup (16 KiB .. 160 KiB). A configuration
 * call, not a run call: it waits for all work on the device (launches in
 * flight read the tables it rewrites), then uploads; graphs captured before it
 * must be captured again. AOL_ERR_UNSUPPORTED when the schedule does not fit; the
 * previous schedule stays in place. Results are identical for every
 * schedule. */
aol_status aol_batch_set_schedule(aol_batch_plan* plan, int32_t seg_reps, int32_t lds_budget);

/* Rebuilds the plan with the current schedule and a new weight (per mille,
 * 250 .. 4000; 1000 after aol_batch_set_schedule) of the int8-tap streams'
 * estimated cost when they and the split-tap streams share one launch: a
 * larger weight gives the int8-tap part more of the device's workgroups. No
 * effect on a plan with one part. A configuration call like
 * aol_batch_set_schedule (graphs must be captured again; AOL_ERR_INVALID for
 * a weight out of range, the previous schedule stays in place). Results are
 * identical for every weight. */
aol_status aol_batch_set_part_weight(aol_batch_plan* plan, int32_t permille);

/* The plan's current schedule as a JSON object (plan-owned string). */
const char* aol_batch_schedule(aol_batch_plan* plan);

/* --------------------------------------------------------------------------
 * General Array-OL repetition with a weighted-sum elementary task.
 *
 * Sec. III-A (tiler footnote): a tiler cuts the pattern of repetition r out of
 * an array as element i of the pattern = array[(origin + paving.r +
 * fitting.i) mod array_shape], component-wise with a non-negative modulus.
 * aol_wsum computes, for every r of the repetition space,
 *
 *   out[(o' + P'.r) mod S'] = sum_i w[i] * in[(o + P.r + F.i) mod S]
 *
 * in float32 (weights and data float32, fused multiply-adds; a plan may sum
 * the pattern grouped by the reads neighbouring points share, so the
 * rounding can differ from a sum in pattern order, always within float32's
 * bound for npat terms). Arrays are dense row-major float32 buffers owned by
 * the caller. paving is array_rank x rep_rank, fitting array_rank x pat_rank,
 * both as [array dim][other dim]; unused entries are ignored. The output
 * tiler must have a single-element pattern (pat_rank 0) and the same
 * repetition space, and must write every output element exactly once: this
 * is checked at plan creation (AOL_ERR_INVALID otherwise). Limits: ranks <= 4,
 * arrays below 2^31 elements, at most 64 pattern elements.
 * ------------------------------------------------------------------------ */
typedef struct aol_tiler {
  int32_t array_rank;
  int32_t rep_rank;
  int32_t pat_rank;
  int32_t reserved;
  int64_t array_shape[4];
  int64_t rep_shape[4];
  int64_t pat_shape[4];
  int64_t origin[4];
  int64_t paving[4][4];
  int64_t fitting[4][4];
} aol_tiler;

typedef struct aol_wsum_plan aol_wsum_plan;

/* weights: host, prod(in->pat_shape) float32 in row-major pattern order;
 * copied into the plan. */
aol_status aol_wsum_plan_create(const aol_tiler* in, const aol_tiler* out, const float* weights,
                                aol_wsum_plan** plan);
/* d_in: the input array (prod(in->array_shape) floats); d_out: the output
 * array (prod(out->array_shape) floats). Enqueue only. */
aol_status aol_wsum_run(aol_wsum_plan* plan, const float* d_in, float* d_out, hipStream_t stream);
aol_status aol_wsum_plan_destroy(aol_wsum_plan* plan);

/* One-shot form of the above: validates both tilers (the bijection check of a
 * non-identity output tiler walks the repetition space on the host) and
 * enqueues the launch on stream. The weights travel in the kernel arguments,
 * so nothing is allocated on the device; same limits and errors as
 * aol_wsum_plan_create and aol_wsum_run. */
aol_status aol_weighted_sum_f32(const aol_tiler* in, const aol_tiler* out, const float* weights, const float* d_in,
                                float* d_out, hipStream_t stream);

/* --------------------------------------------------------------------------
 * General Array-OL repetition with a linear integer elementary task (uint8).
 *
 * Sec. III: the application takes 24-bit RGB frames apart into colour
 * components, filters them and composes the output frame; Sec. III-A: every
 * step is a repetitive task with an input and an output tiler. For every
 * point r of the repetition space
 *
 *   x[i] = in[(o + P.r + F.i) mod S]                   (input pattern, row-major)
 *   y[j] = clamp(floor((sum_i W[j][i] * x[i] + bias[j] + 128) / 256), 0, 255)
 *   out[(o' + P'.r + F'.j) mod S'] = y[j]              (output pattern, row-major)
 *
 * computed exactly (int32 sums). With three-byte patterns this converts
 * interleaved RGB to planar colour components and back (the composition of
 * the frame); with a T x T input pattern and a p x p output pattern it is a
 * non-separable 2-D filter with several outputs per repetition.
 * weights: host, int16 [n_out][n_in] (n_in = prod(in->pat_shape) <= 1024,
 * n_out = prod(out->pat_shape) <= 16); bias: host int32 [n_out] or NULL; both
 * copied into the plan. Both tilers share the repetition space (at most
 * 2^31 - 1 points); arrays are dense row-major uint8 below 2^31 elements.
 * Plan creation checks that the output tiler writes every element of its
 * array exactly once (walking the repetition space on the host;
 * AOL_ERR_INVALID otherwise) and that no sum can leave int32
 * (AOL_ERR_UNSUPPORTED).
 * ------------------------------------------------------------------------ */
typedef struct aol_linear_plan aol_linear_plan;

aol_status aol_linear_plan_create(const aol_tiler* in, const aol_tiler* out, const int16_t* weights,
                                  const int32_t* bias, aol_linear_plan** plan);
/* d_in: prod(in->array_shape) bytes; d_out: prod(out->array_shape) bytes; must
 * not alias. Any alignment; with both pointers 16-byte aligned, plans with
 * small patterns (at most 32 input elements, positive strides between
 * consecutive points of the last repetition dim) stage their rows through
 * LDS with 16-byte accesses (same results). Enqueue only. */
aol_status aol_linear_run(aol_linear_plan* plan, const uint8_t* d_in, uint8_t* d_out, hipStream_t stream);
aol_status aol_linear_plan_destroy(aol_linear_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* AOLMI_H */
