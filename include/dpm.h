/*
 * libdpm -- 3D geometric moments of uint8/uint16 volumes on AMD Instinct MI355X
 * (gfx950) with the Discrete Projection Moment method of Diggin & Diggin,
 * "Fast 3D Image Moments" (arXiv 2012.08099).
 *
 * What is computed (Section 1, eq. 2):
 *     M_pqr = sum_{x,y,z} V(x,y,z) x^p y^q z^r,   0 <= x < L, 0 <= y < M, 0 <= z < N,
 * for every p+q+r <= max_order (0 <= max_order <= 16), with 0^0 = 1.
 *
 * How (Section 3): one pass over the volume forms max_order+1 integer projection
 * images I_d(i, y) = sum over alpha_d x + beta_d z = i of V (eq. 4; the directions
 * (1,0), (0,1), (1,1), (1,-1) are eqs. 5, 6, 8, 9 and the rest are the further
 * aligned projections listed after eq. 9); the 2D power moments of every image are
 * taken (eq. 1); the 3D moments are recovered from them by the recombination of
 * Section 3.2 (eqs. 10-16, generalised to any order).  All arithmetic after the
 * volume read is exact integer arithmetic; orders <= 4 are returned as exact 128-bit
 * integers and every order as the nearest FP64 value of the exact integer.
 *
 * Volume layout: contiguous V[z][y][x] (x fastest), element type uint8 or uint16,
 * resident in device memory.  dims = {L, M, N} = {X, Y, Z} extents.
 *
 * Moment order in every output array ("graded order"): p+q+r ascending; within one
 * total order p descending, then q descending:
 *     M000; M100 M010 M001; M200 M110 M101 M020 M011 M002; ...
 *
 * Conventions for every function below:
 *   - return 0 (DPM_OK) on success or a negative dpm_status; never throw or abort;
 *   - "device pointer" = memory from hipMalloc (or torch) on the current device;
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *   - the library keeps no caller pointer after a call (async: after the stream work
 *     it enqueued has finished);
 *   - calls that enqueue on the same stream are ordered; calls on different streams
 *     that pass their own workspace must pass different ones (calls that use the
 *     library-owned workspace are ordered by the library, see dpm_moments_async).
 */
#ifndef DPM_H
#define DPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DPM_OK = 0,
    DPM_EINVAL = -1,   /* null pointer, dim <= 0, unknown dtype, order outside [0,16], bad size */
    DPM_ERANGE = -2,   /* volume too large for the exact integer widths the library provides */
    DPM_ENOMEM = -3,   /* workspace too small, or device/host allocation failed              */
    DPM_EDEVICE = -4,  /* a HIP runtime error; see dpm_last_device_error()                   */
    DPM_ENOTSUP = -5   /* valid request the library does not implement                       */
} dpm_status;

typedef enum { DPM_U8 = 1, DPM_U16 = 2 } dpm_dtype;

/* Two's complement signed 128-bit integer, little-endian words. */
typedef struct {
    uint64_t lo;
    int64_t hi;
} dpm_i128;

/* Result buffers (caller-owned; host or device memory depending on the call).
 *   exact: dpm_num_moments(min(max_order, 4)) entries -- orders 0..4, exact;
 *          may be NULL if not wanted.
 *   fp64:  dpm_num_moments(max_order) entries -- every order, each the FP64 value
 *          nearest to the exact integer moment (ties to even); may be NULL. */
typedef struct {
    dpm_i128 *exact;
    double *fp64;
} dpm_out;

/* Number of moments with p+q+r <= max_order: (K+1)(K+2)(K+3)/6; -1 if K outside [0,16]. */
int dpm_num_moments(int max_order);

/* Graded-order position of (p,q,r); -1 if any index is negative or p+q+r > 16. */
int dpm_moment_index(int p, int q, int r);

/* Static description of an error code. */
const char *dpm_strerror(int status);

/* hipError_t of the most recent DPM_EDEVICE on this thread (0 if none). */
int dpm_last_device_error(void);

/* Projection direction d (0 <= d <= 16) of the fixed family used for order
 * max_order = d and above: image d sums V along alpha x + beta z = const. */
int dpm_direction(int d, int *alpha, int *beta);

/* Width of projection image d for a volume of the given dims:
 * alpha (L-1) + |beta| (N-1) + 1; 0 on invalid input. */
int64_t dpm_image_width(const int64_t dims[3], int d);

/* Device workspace needed by dpm_moments_async for this request (bytes); 0 if the
 * request is invalid. */
size_t dpm_workspace_bytes(const int64_t dims[3], dpm_dtype dtype, int max_order);

/* Blocking convenience call.  volume: device pointer.  out->exact / out->fp64: HOST
 * memory.  Uses a library-owned workspace (cached per device, freed by dpm_release). */
int dpm_moments(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                dpm_out *out);

/* Stream-ordered call.  volume, out_device->exact/fp64 and workspace are device
 * pointers; workspace must hold dpm_workspace_bytes() bytes, or be NULL to use the
 * library-owned workspace of this device.  That workspace is shared by every call that
 * brings none (dpm_moments, dpm_features, dpm_project_images, dpm_moments_from_images
 * and this call with NULL): the library makes each such call's stream wait, on the
 * device, for the work of the previous one (an event recorded after it), so calls on
 * different streams never overlap on it -- they run one after another.  Returns after
 * enqueueing; results are valid once `stream` reaches this point.
 * Graph capture: with a caller workspace, and once an eager call of the same dims, dtype
 * and order has run on the device (it builds the device tables), the call enqueues
 * kernels only -- no allocation, no memset, every byte it reads written first -- so a
 * caller may capture it into a HIP graph and replay it (new voxels in place included). */
int dpm_moments_async(const void *volume, const int64_t dims[3], dpm_dtype dtype,
                      int max_order, const dpm_out *out_device, void *workspace,
                      size_t ws_bytes, void *stream);

/* ---- allocation-free variant of dpm_moments_async ------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, result and stream
 * semantics as dpm_moments_async, but the workspace (and the power table of the
 * matrix-core power sums, rebuilt by a kernel on `stream` at every call) live in a fixed
 * device array of the library, DPM_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, held from the
 * first call until the process ends.  The call allocates and frees nothing (the first
 * call on a device also uploads the constant recombination tables, a copy).
 * Every call on one GPU uses that GPU's single array: calls that overlap on one GPU
 * (different streams, or threads) race and may return wrong results -- order them (one
 * stream, or events).  Nothing in the array needs clearing: every byte the call reads it
 * writes first.
 * Errors: as dpm_moments_async; DPM_ENOMEM if the request needs more than the array
 * (*scratch_needed, if not NULL, then holds the bytes it would need; e.g. 512^3 uint16
 * needs about 16 MB at order 6 and fits up to order 15, while order 16 needs about
 * 70 MiB: use dpm_moments_async with a caller workspace). */
#define DPM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int dpm_moments_noalloc(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                        const dpm_out *out_device, void *stream, size_t *scratch_needed);
/* DPM_NOALLOC_SCRATCH_BYTES, as built into the library. */
size_t dpm_noalloc_scratch_bytes(void);

/* The max_order+1 projection images of Section 3.1 (step 1 of the method), exact
 * int32.  images_device: device pointer to sum_d M * width_d int32 values; image d is
 * stored row-major as [y][i] right after image d-1.  For beta < 0 the column index
 * carries the offset |beta| (N-1) (column x - z + N - 1 for the (1,-1) image, as in
 * the projection pseudo-code of Section 5).  Requires every line sum to fit in
 * 32 bits (else DPM_ERANGE). */
int dpm_project_images(const void *volume, const int64_t dims[3], dpm_dtype dtype,
                       int max_order, int32_t *images_device, void *stream);

/* Moments from supplied projection images instead of a volume (Section 3.2: chosen
 * tomographic projections can stand in for a full reconstruction).  images_device holds
 * the max_order+1 images exactly as dpm_project_images writes them for a volume of dims
 * and dtype (image d = [y][i], M rows of dpm_image_width(dims, d) int32, one after the
 * other; beta < 0 images carry the offset |beta| (N-1)).  The images are read only:
 * every entry must be a line sum of such a volume, 0 <= entry <= vmax * max(L, N)
 * (vmax 255 / 65535), else DPM_ERANGE (the result is then not written).  Blocking; out's
 * arrays are HOST memory as for dpm_moments; uses the library-owned workspace. */
int dpm_moments_from_images(const int32_t *images_device, const int64_t dims[3], dpm_dtype dtype,
                            int max_order, dpm_out *out);

/* ---- the paper's own route (orders <= 4) -----------------------------------------
 * A verification mode that follows the paper literally.  Step 1 forms the five images
 * of Section 3.1 from one pass over the volume:
 *   XY  I(i = x, j = y)          eq. 5   M rows of L
 *   YZ  I(i = y, j = z)          eq. 6   N rows of M
 *   ZX  I(i = z, j = x)          eq. 7   L rows of N
 *   X+Z I(i = x + z, j = y)      eq. 8   M rows of L + N - 1
 *   X-Z I(i = x - z + N - 1, j = y)  eq. 9 (the column of the projection pseudo-code
 *                                   of Section 5), M rows of L + N - 1
 * -- the first three for orders <= 2, four for order 3, all five for order 4.  ZX sums
 * over y while the others sum over z (or x), so no tile of the volume completes every
 * image: each workgroup writes its partial images and a second kernel sums them in a
 * fixed order (the default path's images avoid this; the difference is the extra
 * traffic this mode exists to show).  Step 2 takes each image's 2D moments (eq. 1)
 * from its five 1D integrals of Section 5 (onto the x and y axes, the 45 and 135 degree
 * axes and the arctan(1/2) axis), by the binomial expansion of (a i + b j)^n.  Step 3
 * is eqs. 10-16 -- eqs. 15 and 16 with their left-hand sides exchanged, as the
 * expansion of (x +- z)^3 y requires -- after shifting the X-Z moments to the origin
 * N - 1 (Section 5).  Results are exact: orders <= 4 as int128 and FP64 (nearest).
 *
 * dpm_paper_workspace_bytes: device workspace for a request (0 if invalid or outside
 * the mode's range: max_order > 4, or an image's W + 2 (H - 1) >= 2^15, i.e. dims up to
 * about 8191).  dpm_paper_images: the images only, into images_device (one after the
 * other in the order above, each row-major [j][i], sum of W*H int32).
 * dpm_moments_paper: the moments, stream-ordered, device outputs as dpm_moments_async.
 * Errors: DPM_EINVAL (arguments), DPM_ENOTSUP (max_order > 4), DPM_ERANGE (range),
 * DPM_ENOMEM (workspace smaller than dpm_paper_workspace_bytes). */
size_t dpm_paper_workspace_bytes(const int64_t dims[3], dpm_dtype dtype, int max_order);
int dpm_paper_images(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                     int32_t *images_device, void *workspace, size_t ws_bytes, void *stream);
int dpm_moments_paper(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                      const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream);

/* The default projection images (the family of dpm_project_images) with their 2D moments
 * taken by the 1D-integral route of Section 5 instead of direct power sums (orders <= 4):
 * each image's 1D integrals along (1,0), (0,1), (1,1), (1,-1), (1,2) in its (i, y) plane,
 * their 1D moments about the image's origin, the exact 1D -> 2D inverse, then the
 * recombination of Section 3.2 as in dpm_moments_async.  Same outputs and stream
 * semantics as dpm_moments_async; workspace of dpm_drt_workspace_bytes (0 if invalid
 * or out of range: orders > 4, or an image's width + 2 (M - 1) >= 2^15). */
size_t dpm_drt_workspace_bytes(const int64_t dims[3], dpm_dtype dtype, int max_order);
int dpm_moments_drt(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                    const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream);

/* ---- object features (Section 4, after the moments) ---------------------------
 * From the exact moments of one volume (eq. 2), for every moment of order <= max_order
 * in graded order:
 *   centroid   (x̄, ȳ, z̄) = (M100, M010, M001) / M000;
 *   mu         central moments  mu_pqr = sum V (x - x̄)^p (y - ȳ)^q (z - z̄)^r;
 *   eta        scale-normalised eta_pqr = mu_pqr / mu_000^((p+q+r)/3 + 1);
 *   mu_phys    physical spacing mu'_pqr = alpha^(1+p) beta^(1+q) delta^(1+r) mu_pqr with
 *              (alpha, beta, delta) = spacing (NULL: 1, 1, 1).
 * M000^n mu_pqr (n = p+q+r) is formed as an exact integer on the device, so mu carries
 * no cancellation error: it is the exact rational rounded twice to double (relative
 * error below 2^-51; mu_100 = mu_010 = mu_001 = 0 exactly).  A volume of zero mass
 * gives NaN for the centroid and for every moment of order >= 1 (mu_000 = M000 = 0).  Blocking; volume is a device pointer; out's arrays are HOST
 * memory of dpm_num_moments(max_order) doubles (eta, mu_phys may be NULL).  Uses the
 * library-owned workspace of the device.  DPM_ERANGE if the exact numerators would need
 * more than 1024 bits (orders near 16 of volumes much larger than 512^3). */
typedef struct {
    double centroid[3];
    double *mu;
    double *eta;
    double *mu_phys;
} dpm_features_out;

int dpm_features(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                 const double spacing[3], dpm_features_out *out);

/* ---- batched regions of interest --------------------------------------------
 * Many independent volumes ("ROIs") in one packed device buffer; each ROI is its own
 * volume with its own origin (eq. 2 applied to the ROI).  ROI i starts at byte
 * offset rois[i].offset_bytes of `packed`, holds dims[0]*dims[1]*dims[2] elements of
 * rois[i].dtype in V[z][y][x] order.  Rows start 16-byte aligned and whole rows are
 * readable when (offset_bytes % 16 == 0 and L*elem % 16 == 0); otherwise the ROI is
 * read with narrower loads (correct, slower). */
typedef struct {
    uint64_t offset_bytes;
    int64_t dims[3];
    int32_t dtype; /* dpm_dtype */
    int32_t reserved;
} dpm_roi;

size_t dpm_batched_workspace_bytes(const dpm_roi *rois, int n_rois, int max_order);

/* All ROIs in one launch sequence on `stream`: a prep kernel (per-ROI geometry and
 * work items); a fused kernel in which a workgroup projects a block of 16 y-slices of
 * one ROI (Section 3.1, eq. 4) and takes the exact power sums of the block's image rows
 * without writing them to memory, for every ROI whose block fits its LDS (about 80 KB)
 * when the exact sums fit 128 bits; for the other ROIs (all of them with
 * DPM_BATCH_FUSED=0 in the environment) a projection kernel per (ROI, y) slice that
 * writes the rows and a power-sum kernel over them; one recombination per ROI
 * (Section 3.2).  Both ways give the same integers.  Orders <= 6 (else DPM_ENOTSUP); ROI
 * dims <= 4096, and every ROI's image rows over its whole z range must fit the LDS of
 * one workgroup (160 KB; e.g. a 1 x 1 x 4096 column at order 6 does not), else
 * DPM_ERANGE -- dpm_batched_workspace_bytes then returns 0; such a volume goes through
 * dpm_moments_async, which splits z.  out_device->exact / ->fp64 hold n_rois consecutive
 * result blocks (block i at i * dpm_num_moments(...)); workspace must hold
 * dpm_batched_workspace_bytes() bytes (else DPM_ENOMEM).
 *
 * Repeated calls: when a call repeats an earlier one exactly (same ROI descriptors,
 * order, packed / output / workspace pointers and workspace size, same device), its
 * launch sequence is captured into a hipGraph on the second sighting and replayed from
 * then on, with no host planning and no descriptor upload; the contents of `packed` may
 * change between calls.  Up to 16 graphs are cached, least recently used evicted; they
 * are freed by dpm_release.  Graphs are not used while stage timing is enabled, when
 * the environment sets DPM_NO_GRAPH=1, or for the served loop's batches (they rarely
 * repeat, and a capture allocates synchronously).  A graph whose launch fails is dropped
 * and the call runs without it.  Not safe against concurrent calls that share a
 * workspace. */
int dpm_moments_batched(const void *packed, const dpm_roi *rois, int n_rois, int max_order,
                        const dpm_out *out_device, void *workspace, size_t ws_bytes,
                        void *stream);

/* Number of batched-call graphs currently cached (see dpm_moments_batched). */
int dpm_batched_graph_count(void);

/* Free every library-owned device workspace, cached table and cached graph.  Call it
 * only when no library work is in flight. */
int dpm_release(void);

/* ---- stage timing (tracing) --------------------------------------------------
 * While enabled, every dpm_moments / dpm_moments_async / dpm_moments_batched call
 * records HIP events on its own stream before the projection kernel and after each of
 * the three stages.  dpm_profile_collect waits for the recorded events, returns the summed
 * device time per stage and clears the record.  Event creation happens at record
 * time, so enable this only for measurement (it is host-side overhead, not device
 * work).  Not thread-safe with concurrent callers on different streams. */
typedef struct {
    int32_t calls;
    int32_t reserved;
    double ms_project;    /* projection kernel(s): one pass over the volume       */
    double ms_power;      /* exact power sums of the image rows, y-weighted per tile */
    double ms_combine;    /* tile sums to 2D moments and recombination into 3D   */
    double ms_total;
} dpm_profile;

int dpm_profile_enable(int on);
int dpm_profile_collect(dpm_profile *out);

/* ---- served loop ---------------------------------------------------------------
 * A request server for a stream of independent volumes of mixed sizes: the batched
 * and served workloads of a moment service (the paper computes one volume at a time;
 * every request here is that computation, eq. 2 via Sections 3.1-3.2).
 *
 * The server owns one device arena of `hbm_budget` bytes, `n_streams` HIP streams and
 * a worker thread.  Requests are admitted first come, first served, when their device
 * blocks (copied volume if it arrives in host memory, workspace, device outputs) fit in
 * the arena; a request whose blocks can never fit is refused at submit (DPM_ERANGE).
 * Requests of at most `batch_voxels` voxels and order <= 6 that are waiting together are
 * served by one dpm_moments_batched launch sequence (up to `batch_max` of them);
 * larger ones by dpm_moments_async.  Jobs go to the stream with the fewest jobs in
 * flight.  Results are copied to the caller's host buffers before the completion is
 * reported.
 *
 * Requests of one batched launch have the same order (a batch takes waiting small
 * requests of the first one's order, in arrival order).
 * Ownership: the caller keeps `data` and the output buffers of a request valid until
 * its completion has been returned by dpm_server_poll.  A request's `data` may be host
 * memory (copied to the arena) or device memory on the server's device (read in place;
 * batched requests are copied into a packed arena block first).  Device data must be
 * complete when the server reads it: pass `ready_event` (recorded on the stream that
 * writes it), or finish writing before submitting.
 * Residency: with keep_resident = 1 the request's 2D moments of every side of every
 * projection image (eq. 1 of the images of Section 3.1; 2 (K+1)^3 exact integers) stay in
 * the arena after completion, under the request's tag.  dpm_server_requery recombines
 * them (Section 3.2) for any order <= K without reading the volume again.  Entries are
 * evicted least recently used (a query counts as a use) whenever a request cannot be
 * admitted otherwise, or dropped by dpm_server_release.
 * Thread safety: submit and poll may be called from any threads.
 * Errors: submit returns DPM_EINVAL for a malformed request and DPM_ERANGE if it cannot
 * fit the budget; a request that fails on the device completes with its status. */
typedef struct {
    int32_t device;          /* HIP device ordinal                                      */
    int32_t n_streams;       /* streams used for jobs (>= 1)                            */
    int64_t hbm_budget;      /* bytes of device memory for the arena                    */
    int64_t batch_voxels;    /* requests of at most this many voxels may be batched     */
    int32_t batch_max;       /* most requests in one batched launch                     */
    int32_t max_inflight;    /* most jobs in flight (pinned result slots)               */
} dpm_server_config;

typedef struct dpm_server dpm_server;  /* opaque */

typedef struct {
    const void *data;        /* contiguous V[z][y][x]                                   */
    int32_t data_on_device;  /* 1: device pointer on the server's device, 0: host memory */
    int32_t dtype;           /* dpm_dtype                                               */
    int64_t dims[3];         /* L, M, N                                                 */
    int32_t max_order;       /* 0..16 (batched only when <= 6)                          */
    int32_t keep_resident;   /* 1: keep the request's image moments on the device after
                                completion, for dpm_server_requery (see below)          */
    uint64_t tag;            /* returned with the completion; names a resident entry    */
    double t_arrival_ms;     /* arrival time on the server clock (dpm_server_now_ms);
                                <= 0: the submit time                                  */
    dpm_i128 *exact;         /* host, n_moments(min(K,4)) entries, or NULL              */
    double *fp64;            /* host, n_moments(K) entries, or NULL                     */
    void *ready_event;       /* device data only: a hipEvent_t recorded after the work
                                that writes `data`; the server's stream waits for it
                                before reading.  NULL: `data` is complete at submit.   */
} dpm_request;

typedef struct {
    uint64_t tag;
    int32_t status;          /* DPM_OK or the failure                                   */
    int32_t batched;         /* 1: served in a batched launch                           */
    double t_arrival_ms;     /* server clock                                            */
    double t_start_ms;       /* first device work issued                                */
    double t_done_ms;        /* results in the caller's buffers                         */
} dpm_completion;

typedef struct {
    int64_t submitted, completed, batched_jobs, single_jobs;
    int64_t arena_bytes, arena_peak_used;
    int32_t pending, inflight;
    int64_t resident, resident_bytes, evictions;  /* resident entries (see requery) */
} dpm_server_stats;

/* Milliseconds on the server clock (monotonic). */
double dpm_server_now_ms(void);
int dpm_server_create(const dpm_server_config *cfg, dpm_server **out);
int dpm_server_submit(dpm_server *s, const dpm_request *req);
/* Up to `max` completions; waits up to wait_ms (0: no wait) for the first one.  Returns
 * the number written, or a negative status. */
int dpm_server_poll(dpm_server *s, dpm_completion *out, int max, int wait_ms);
int dpm_server_stats_get(dpm_server *s, dpm_server_stats *out);
/* Load generator: submits reqs[0..n) in order, each at its t_arrival_ms on the server
 * clock (sleeping, then spinning for the last 0.2 ms), and returns once all are
 * submitted (or the first failing submit's status).  Arrival times must not decrease. */
int dpm_server_replay(dpm_server *s, const dpm_request *reqs, int n);
/* Moments of order <= max_order (<= the request's order) of a resident request, from its
 * resident image moments: exact / fp64 are HOST buffers as in dpm_request (either may be
 * NULL).  Blocking (runs on a stream of the server).  DPM_EINVAL if `tag` is not resident
 * (never kept, evicted or released) or max_order exceeds its order. */
int dpm_server_requery(dpm_server *s, uint64_t tag, int max_order, dpm_i128 *exact, double *fp64);
/* Drop a resident entry (DPM_EINVAL if `tag` is not resident). */
int dpm_server_release(dpm_server *s, uint64_t tag);
/* Waits for every submitted request, then frees the server (completions not yet
 * polled are dropped). */
int dpm_server_destroy(dpm_server *s);

/* ---- introspection used by the host-side tests ------------------------------ */

/* Exact recombination weight of Section 3.2 generalised: for total x-z degree k,
 *   M_{p, q, k-p} = sum_{d<=k} num[p][d] * m_d / den[p]
 * where m_d is the degree-(k, q) 2D moment of image d about its true origin.
 * Writes num (int64) and den (uint64, > 0) for one (k, p, d). */
int dpm_recomb_weight(int k, int p, int d, int64_t *num, uint64_t *den);

/* Planning summary for a request (host logic only; no device work). */
typedef struct {
    int32_t n_dirs;        /* max_order + 1                                   */
    int32_t n_groups;      /* launches of the projection kernel               */
    int32_t n_items;       /* workgroups per launch (y-slices x z-splits)     */
    int32_t z_splits;      /* z-splits per y-slice                            */
    int32_t limbs_slice;   /* 32-bit limbs of per-slice partial sums          */
    int32_t limbs_moment;  /* 32-bit limbs of 2D moments and recombination    */
    int32_t bits_slice;    /* bound on partial sums (bits incl. sign)         */
    int32_t bits_moment;   /* bound on recombination numerators (bits)        */
    int64_t lds_bytes;     /* LDS per projection workgroup (largest group)    */
    int64_t workspace;     /* bytes                                           */
    int32_t power_tiles;   /* workgroups of the power-sum kernel              */
    int32_t power_chunk;   /* steps of 64 values of a per power tile (0: rows) */
    int32_t proj_waves;    /* waves per workgroup of the first projection launch */
    int32_t reserved;
} dpm_plan_info;

int dpm_plan(const int64_t dims[3], dpm_dtype dtype, int max_order, dpm_plan_info *info);

/* ---- tuning ---------------------------------------------------------------------
 * Per-shape overrides of three planner choices, installed by an autotuner (the Python
 * package's `autotune` module times the candidates through dpm_moments_async and
 * installs the fastest).  Both change how the work is split, never the result.
 *   z_splits:    work items per y-slice (each projection workgroup takes a z range);
 *                0 = the planner's choice.
 *   power_chunk: steps of 64 values of a per power-sum tile on the matrix cores;
 *                0 = the planner's choice, -1 = whole rows.
 *   waves:       waves per projection workgroup of the first direction group when
 *                whole rows are loaded: 0 = the planner's choice (8), 4 or 8.
 * An override applies to every later plan of exactly these dims, dtype and order, and
 * to the workspace size reported for them (query dpm_workspace_bytes after setting
 * it).  The environment overrides DPM_ZSPLITS / DPM_PW_KCHUNK take precedence.
 * t == NULL removes the override of this shape; dpm_tune_clear removes all.
 * Errors: DPM_EINVAL for bad dims, dtype, order, z_splits outside [0, 4096],
 * power_chunk outside [-1, 4096] or waves not 0, 4 or 8. */
typedef struct {
    int32_t z_splits;
    int32_t power_chunk;
    int32_t waves;
    int32_t reserved;
} dpm_tuning;

int dpm_tune_set(const int64_t dims[3], dpm_dtype dtype, int max_order, const dpm_tuning *t);
int dpm_tune_clear(void);

/* Override of the batched call's geometry for batches of order max_order (0-6), for
 * callers that measured a better one (the package's `autotune.tune_batched` times the
 * candidates through dpm_moments_batched and installs the fastest).  It changes how the
 * work is split, never the result.
 *   fused:   0 = the planner's routing (every ROI whose block of 16 slices fits the fused
 *            kernel takes it); -1 = every ROI takes the separate kernels (rows in the
 *            workspace).
 *   units:   projection units per sub-row that grouping slices per wave aims at;
 *            0 = the planner's choice (2), else 1-16.
 *   max_spw: most slices one wave projects together; 0 = the planner's choice (4), or
 *            1, 2 or 4.
 * The override applies to every later batched call and workspace query of that order
 * (query dpm_batched_workspace_bytes after setting it: the separate kernels need rows in
 * the workspace); cached graphs of earlier calls are not replayed after a change.
 * Calls already enqueued keep their plan; set it before serving rather than during.
 * t == NULL removes the override of that order.
 * Errors: DPM_EINVAL for an order outside [0, 6], fused not 0 or -1, units outside
 * [0, 16] or max_spw not 0, 1, 2 or 4. */
typedef struct {
    int32_t fused;
    int32_t units;
    int32_t max_spw;
    int32_t reserved;
} dpm_batch_tuning;

int dpm_batch_tune_set(int max_order, const dpm_batch_tuning *t);

#ifdef __cplusplus
}
#endif
#endif /* DPM_H */
