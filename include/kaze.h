/*
 * kaze.h - C ABI of the MI355X (gfx950) KAZE nonlinear scale-space library.
 *
 * The library computes the detector half of KAZE feature extraction
 * (Ramkumar B et al., "GPGPU Acceleration of the KAZE Image Feature
 * Extraction Algorithm", arXiv 1706.06750):
 *
 *   - the nonlinear scale space of Sec. II-A (Eqs. 1-7): Gaussian
 *     pre-smoothing with sigma0, the contrast factor k from the gradient
 *     histogram (Sec. III-A), the Perona-Malik conductivity (Eqs. 2-3), and
 *     one semi-implicit step (Eq. 4) per level, evaluated by additive
 *     operator splitting with tridiagonal solves along every row and every
 *     column and zero-flux (Neumann) boundaries;
 *   - the scale-normalised Hessian determinant of every level (Eq. 8);
 *   - the 3x3x3 non-maximum suppression of Sec. II-B.
 *
 * Conventions shared by every entry point:
 *   - Pointers marked (device) are HIP device pointers on the current
 *     device; pointers marked (host) are read during the call only.
 *   - Images and levels are float32, row-major.  `levels` and `det` hold
 *     N = octaves*sublevels planes of H rows of W floats, densely packed.
 *   - Calls are asynchronous: they validate their arguments, enqueue work on
 *     `stream` (a hipStream_t; NULL is the null stream) and return without
 *     synchronising.  Argument errors are returned synchronously and
 *     enqueue nothing.  A failed HIP launch returns KAZE_ERR_HIP.
 *   - The caller owns every buffer.  The library allocates no device memory:
 *     scratch lives in a caller-provided workspace of
 *     kaze_workspace_bytes() bytes (256-byte aligned).  Two calls that
 *     share a workspace must be ordered on the same stream.
 *   - Size limits: 8 <= W, H <= 4096, N <= 64, Gaussian radius ceil(3 sigma)
 *     <= 16 for sigma0 and <= 4 for sigma_cond, Scharr step of Eq. 8 <= 8.
 *   - Nothing throws across the ABI.
 */
#ifndef KAZE_H
#define KAZE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KAZE_OK = 0,
    KAZE_ERR_INVALID_ARG = -1,  /* a pointer, size or parameter is invalid   */
    KAZE_ERR_WORKSPACE = -2,    /* workspace missing, misaligned or too small */
    KAZE_ERR_HIP = -3,          /* a HIP launch or runtime call failed        */
    KAZE_ERR_UNSUPPORTED = -4   /* valid but outside the supported limits     */
} kaze_status;

/* Perona-Malik conductivity functions of Eq. 3. */
typedef enum { KAZE_G1 = 1, KAZE_G2 = 2 } kaze_diffusivity;

/* How each level is reached from the one before, with the conductivity of
 * the level before held fixed:
 *   KAZE_AOS  one semi-implicit step of Eq. 4 (additive operator splitting);
 *   KAZE_FED  one fast-explicit-diffusion cycle of Eq. 5 (see
 *             kaze_fed_schedule). */
typedef enum { KAZE_AOS = 0, KAZE_FED = 1 } kaze_scheme;

/* Cross-level window of the extrema test (Sec. II-B, Sec. III-B, Sec. IV):
 *   KAZE_WINDOW_3X3    the "approximate" test: 3x3 in levels i-1 and i+1;
 *   KAZE_WINDOW_SIGMA  the "exact" test: a square window of side 2h+1 in
 *                      levels i-1 and i+1, the odd side nearest sigma_i
 *                      (h = max(1, round((sigma_i - 1)/2)), half up),
 *                      clipped at the image border. */
typedef enum { KAZE_WINDOW_3X3 = 0, KAZE_WINDOW_SIGMA = 1 } kaze_extrema_window;

/* Largest histogram of the contrast factor k (kaze_params.k_bins). */
#define KAZE_MAX_K_BINS 4096

/*
 * Parameters of the method (host struct, read during the call only).
 * kaze_default_params() fills the values used throughout: sigma0 = 1.6,
 * 4 octaves x 4 sublevels, sigma_cond = 1.0, g2, k at the 70th percentile
 * of a 300-bin gradient histogram, detector threshold 0.001, AOS steps.
 */
typedef struct {
    int    octaves;        /* O of Eq. 6                                        */
    int    sublevels;      /* S of Eq. 6                                        */
    double sigma0;         /* base scale of Eq. 6; pre-smoothing width          */
    double sigma_cond;     /* Gaussian width before the conductivity gradient   */
    int    diffusivity;    /* KAZE_G2 (default) or KAZE_G1, Eq. 3               */
    int    k_bins;         /* histogram bins, 1..KAZE_MAX_K_BINS                */
    double k_percentile;   /* quantile of the gradient histogram, [1e-6, 1]     */
    double k_override;     /* > 0: use this contrast factor, skip the histogram */
    double det_threshold;  /* detector threshold of Sec. II-B (compared in FP32) */
    int    scheme;         /* KAZE_AOS (default) or KAZE_FED                     */
    int    extrema_window; /* KAZE_WINDOW_3X3 (default) or KAZE_WINDOW_SIGMA     */
    int    substeps;       /* steps per level, 1..64 (default 1): the step of
                            * length tau_i is split into this many equal steps
                            * (AOS steps or FED cycles), each with the
                            * conductivity of its own starting image          */
} kaze_params;

/* One detected extremum: pixel position, level index and det response. */
typedef struct {
    int   x;
    int   y;
    int   level;
    float response;
} kaze_keypoint;

/* A refined extremum (kaze_refine_keypoints). */
typedef struct {
    float x, y;        /* sub-pixel position                                   */
    int   level;
    float response;    /* value of the fitted quadratic at its maximum         */
    float edge_ratio;  /* Tr(H)^2 / Det(H) of Eqs. 10-12; +inf if Det(H) <= 0   */
    int   kept;        /* 1: a maximum, edge_ratio below (r+1)^2/r, |offset| <= 1 */
} kaze_keypoint_refined;

/* Fills *p with the defaults listed above.  Returns KAZE_ERR_INVALID_ARG
 * for a NULL pointer. */
kaze_status kaze_default_params(kaze_params* p);

/* Number of scale levels N = octaves * sublevels (Eq. 6), or a negative
 * kaze_status if *p is invalid. */
int kaze_num_levels(const kaze_params* p);

/*
 * Per-level schedule of Eqs. 6-7 and Eq. 8 (host arrays of length N, any of
 * them may be NULL): sigma_i, evolution time t_i = sigma_i^2/2, the step
 * tau_i = t_i - t_{i-1} into level i (tau_0 = 0), the normalised scale
 * sigma_i / 2^o_i and the Scharr step round(sigma_i / 2^o_i).
 */
kaze_status kaze_schedule(const kaze_params* p, double* sigma, double* t,
                          double* tau, double* sigma_norm, int* deriv_step);

/* Workspace bytes that kaze_build_scale_space needs for a W x H image, or 0
 * if the arguments are invalid. */
size_t kaze_workspace_bytes(int W, int H, const kaze_params* p);

/*
 * Nonlinear scale space (Sec. II-A, Sec. III-A).
 *   img      (device) W x H float32 image, row pitch ld_img >= W floats.
 *   levels   (device) output, N x H x W float32: level 0 is G_sigma0 * img,
 *            level i >= 1 is one AOS step of Eq. 4 (or one FED cycle of
 *            Eq. 5, p->scheme) from level i-1 with tau_i, conductivity
 *            computed from level i-1.
 *   k_out    (device) output, 1 float32: the contrast factor used (the
 *            histogram quantile of Sec. III-A, or k_override).
 *   ws       (device) workspace of at least kaze_workspace_bytes(W, H, p)
 *            bytes, 256-byte aligned; its contents on entry are ignored.
 *   stream   hipStream_t to enqueue on.
 * The input image must not alias levels or the workspace.
 */
kaze_status kaze_build_scale_space(const float* img, int W, int H, int ld_img,
                                   const kaze_params* p, float* levels,
                                   float* k_out, void* ws, size_t ws_bytes,
                                   void* stream);

/* Bytes of the device-resident scratch of kaze_build_scale_space_noalloc
 * (64 MiB per GPU): enough for the default parameters up to 3840 x 2160,
 * or up to about 2560 x 1600 with FED or sub-steps. */
#define KAZE_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * kaze_build_scale_space without a workspace argument, for callers that
 * cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Arguments, outputs and results
 * are those of kaze_build_scale_space (the same kernels on the same scratch
 * layout, bit for bit); the scratch is a static device array of
 * KAZE_NOALLOC_SCRATCH_BYTES that the library's code object holds on every
 * GPU it runs on until the process ends.  Its address is looked up on the
 * current device the first time the call runs there; the call itself
 * allocates and frees nothing.
 *   Limits: returns KAZE_ERR_UNSUPPORTED, before enqueuing anything, when
 *   kaze_workspace_bytes(W, H, p) exceeds KAZE_NOALLOC_SCRATCH_BYTES.
 *   Concurrency: every call on one GPU uses that GPU's one scratch array,
 *   which keeps the last call's contents (nothing in it needs to start at
 *   zero).  Calls that can overlap on one GPU -- on different streams, or
 *   from different threads without ordering -- race on it; order them on
 *   one stream.
 */
kaze_status kaze_build_scale_space_noalloc(const float* img, int W, int H, int ld_img,
                                           const kaze_params* p, float* levels,
                                           float* k_out, void* stream);

/*
 * Conductivity of Eqs. 2-3 for one image and a given contrast factor:
 *   g = 1/(1 + |grad L_s|^2/k^2)  (KAZE_G2)  or  exp(-|grad L_s|^2/k^2) (KAZE_G1),
 * where grad is the 3x3 Scharr gradient (divided by 32) of
 * L_s = G_sigma_cond * L, both with half-sample reflection at the border.
 *   L        (device) input, W x H float32, row pitch W.
 *   k        contrast factor, > 0.
 *   g        (device) output, W x H float32; must not alias L.
 * g equals, bit for bit, the conductivity that the AOS steps of
 * kaze_build_scale_space form internally from the same level and k.
 */
kaze_status kaze_conductivity(const float* L, int W, int H, const kaze_params* p,
                              double k, float* g, void* stream);

/*
 * One AOS step of Eq. 4 with a given conductivity:
 *   L_next = L + (delta_x + delta_y)/2,
 *   (I - 2 tau A_l(g)) delta_l = 2 tau A_l(g) L   for l = rows, columns,
 * A_l having couplings (g_j + g_k)/2 between neighbours along the line and
 * no flux across the image border.
 *   L, g     (device) inputs, W x H float32.
 *   tau      step size, > 0.
 *   L_next   (device) output, W x H float32; must not alias L, g or ws.
 *   ws       (device) workspace of kaze_workspace_bytes(W, H, p) bytes
 *            (any valid p), 256-byte aligned.
 */
kaze_status kaze_aos_step(const float* L, const float* g, int W, int H, double tau,
                          float* L_next, void* ws, size_t ws_bytes, void* stream);

/*
 * Step sizes of one fast-explicit-diffusion cycle of total time T (Eq. 5),
 * as used for every level when p->scheme is KAZE_FED (host, double):
 *   n = the smallest cycle length with tau_max (n^2 + n) / 3 >= T, where
 *       tau_max = 1/4 is the stability limit of the explicit 5-point step
 *       with unit grid spacing and g <= 1;
 *   tau_j = tau_max / (2 cos^2(pi (2j + 1) / (4n + 2))), j = 0..n-1, scaled
 *       so that they sum to T;
 *   order: the steps are applied as j = kappa * i mod n, i = 0..n-1, with
 *       the kappa coprime to n (smallest on ties) that minimises
 *       max_i (max|prefix product| * max|suffix product|) of the step
 *       factors (1 + tau_j mu) over mu in [-8, 0] (2001 points), which
 *       bounds how much rounding errors can grow inside the cycle.
 * Returns n (or a negative kaze_status for T <= 0 or not finite) and, if
 * tau is not NULL and capacity >= n, writes the n step sizes in application
 * order.
 */
int kaze_fed_schedule(double T, double* tau, int capacity);

/*
 * One FED cycle of total time T with a given conductivity (the counterpart
 * of kaze_aos_step): n explicit steps
 *   L <- L + tau_j sum_q (g_p + g_q)/2 (L_q - L_p)
 * over the 4-neighbours q of every pixel p, none across the image border,
 * with the step sizes of kaze_fed_schedule(T).
 *   L, g     (device) inputs, W x H float32.
 *   T        cycle time, > 0.
 *   L_next   (device) output, W x H float32; must not alias L, g or ws.
 *   ws       (device) workspace of kaze_workspace_bytes(W, H, p) bytes for a
 *            p with scheme KAZE_FED, 256-byte aligned.
 */
kaze_status kaze_fed_cycle(const float* L, const float* g, int W, int H, double T,
                           float* L_next, void* ws, size_t ws_bytes, void* stream);

/*
 * Detector response of Eq. 8 for every level:
 *   det_i = sigma_n^2 (L_xx L_yy - L_xy^2), sigma_n = sigma_i / 2^o_i,
 * with second derivatives formed by applying the concatenated Scharr filter
 * of step round(sigma_n) twice (L_xx = D_x D_x L, L_yy = D_y D_y L,
 * L_xy = D_y D_x L), each derivative image extended by half-sample
 * reflection at the border.
 *   levels   (device) input, N x H x W float32.
 *   det      (device) output, N x H x W float32; must not alias levels.
 */
kaze_status kaze_detector_response(const float* levels, int W, int H,
                                   const kaze_params* p, float* det,
                                   void* stream);

/*
 * Non-maximum suppression (Sec. II-B): (x, y, i) is reported iff
 * 1 <= i <= N-2, 1 <= x <= W-2, 1 <= y <= H-2, det_i(x, y) > det_threshold,
 * det_i(x, y) is strictly greater than its 8 neighbours in level i and than
 * every response of levels i-1 and i+1 in the cross-level window of
 * p->extrema_window (3x3: the 26 neighbours of the 3x3x3 block).
 *   det      (device) input, N x H x W float32.
 *   kps      (device) output array of `capacity` keypoints (may be NULL if
 *            capacity is 0).  Only min(*count, capacity) entries are
 *            written, in unspecified order.
 *   count    (device) output, 1 int: the number of extrema found, which may
 *            exceed capacity.  It is reset by the call itself.
 */
kaze_status kaze_find_extrema(const float* det, int W, int H,
                              const kaze_params* p, kaze_keypoint* kps,
                              int capacity, int* count, void* stream);

/*
 * Batches (many images of different sizes in one launch per phase).
 *
 * One image of a batch.  All pointers are (device); det/count may be NULL
 * (then for every image of the batch), which skips the detector response
 * and extrema.
 */
typedef struct {
    const float* img;      /* W x H float32 input, row pitch ld_img          */
    int W, H, ld_img;
    float* levels;         /* N x H x W output                               */
    float* det;            /* N x H x W output, or NULL                      */
    float* k;              /* 1 float output: the contrast factor used       */
    kaze_keypoint* kps;    /* keypoint output (NULL with capacity 0)         */
    int capacity;
    int* count;            /* 1 int output: extrema found, or NULL           */
} kaze_image_desc;

/* Number of AOS launch shapes. */
#define KAZE_AOS_SHAPES 6

/*
 * Launch shape of the row/column solves of the AOS steps (Eq. 4): the blocks
 * of the reduction and recovery launches cover tiles of 60 x ty pixels, row
 * lines are cut into chunks of rc pixels and column lines into chunks of cc,
 * and the interface system of every line is solved with m chunks per lane.
 * With l = 2 lanes per chunk each chunk is reduced and recovered in two
 * halves on a lane pair (the halves meet in a 2x2 system of their middle
 * unknowns); with l = 1 one lane walks the whole chunk.
 *
 *   shape   tile    rc   cc   m   l
 *     0     60x32   30   32   4   2
 *     1     60x32   30   32   8   2
 *     2     60x64   30   32   4   1
 *     3     60x64   30   32   8   1
 *     4     60x64   60   64   4   2
 *     5     60x64   60   64   8   2
 *
 * rc, cc, m and l fix the elimination order, so the shapes agree with each
 * other to FP32 rounding; a shape's results do not depend on the images
 * batched with it.  Every shape fits every image size.
 * aos_shape -1 selects the default: shape 1 when the interface launch has
 * at least 1024 wavefronts at m = 8 over all images of the call, else shape
 * 0 (single-image calls use the same rule).
 */
typedef struct {
    int aos_shape;
} kaze_batch_config;

/* Tile width and height, chunk lengths, interface chunks per lane and sweep
 * lanes per chunk of a shape (host outputs, any may be NULL);
 * KAZE_ERR_INVALID_ARG for a shape outside [0, KAZE_AOS_SHAPES). */
kaze_status kaze_aos_shape_info(int shape, int* tile_w, int* tile_h, int* row_chunk,
                                int* col_chunk, int* iface_m, int* chunk_lanes);

typedef struct kaze_batch kaze_batch;  /* opaque plan */

/* Workspace bytes of a batch for the given shape (cfg NULL or shape -1: the
 * maximum over every shape that fits all images); 0 if invalid. */
size_t kaze_batch_workspace_bytes(const kaze_image_desc* images, int n,
                                  const kaze_params* p,
                                  const kaze_batch_config* cfg);

/*
 * Builds a plan for the images (host array of n descriptors, copied): the
 * per-image descriptor tables and the tile, line and block work lists are
 * written into ws (synchronously), and the whole sequence -- base image,
 * contrast factor, N-1 AOS steps, detector response, extrema, each phase
 * one launch over all images -- is captured once into a hipGraph.  The plan
 * reads and writes the buffers named in the descriptors every time it runs;
 * ws must stay allocated and untouched while the plan exists.
 */
kaze_status kaze_batch_create(const kaze_image_desc* images, int n,
                              const kaze_params* p,
                              const kaze_batch_config* cfg, void* ws,
                              size_t ws_bytes, kaze_batch** out);

/*
 * Properties of a created batch: the AOS tile shape in use and the number of
 * levels whose detector response runs inside the level segment of a run
 * (the one kaze_profile_begin("aos_reduce") brackets), on a second stream
 * beside the steps: all N for batches of 32 Mpx and more with a detector
 * (level by level, in graph and eager runs), else 0 (the detector runs
 * after the steps).
 */
kaze_status kaze_batch_properties(const kaze_batch* b, int* aos_shape,
                                  int* det_levels_in_segment);

/* Enqueues one run of the plan on stream: three graph launches (base image
 * and contrast factor; the AOS steps; detector response and extrema), or
 * with eager != 0 the same kernel launches issued one by one (faster on
 * this runtime for one 1920x1200 image: graph replay adds about 20 us per
 * run).  The detector forks onto the plan's second stream as the
 * properties below describe, ordered through events.  Runs that share a plan must be
 * ordered on one stream.  Under kaze_profile_begin with aos_reduce listed,
 * a run records one event pair around its AOS-step segment (and none
 * around the single launches inside it). */
kaze_status kaze_batch_run(kaze_batch* b, int eager, void* stream);

kaze_status kaze_batch_destroy(kaze_batch* b);

/*
 * Autotuner: for every launch shape (tile height, chunk lengths, interface
 * chunks per lane) that fits all images, builds the plan in ws (sized for
 * the maximum), times `reps` graph launches on stream, and returns the
 * fastest shape in *best and, if ms_per_shape is not NULL, the mean
 * milliseconds per run of each of the KAZE_AOS_SHAPES shapes (-1 where it
 * does not fit).  Synchronises the stream.
 */
kaze_status kaze_batch_autotune(const kaze_image_desc* images, int n,
                                const kaze_params* p, void* ws, size_t ws_bytes,
                                int reps, void* stream, kaze_batch_config* best,
                                double* ms_per_shape);

/*
 * Sub-pixel refinement and edge test of extrema (Sec. II-B, Eqs. 9-12).
 * For keypoint i (i < min(*count, capacity)) the detector responses of its
 * level in the 3x3 window around it are fitted in the least-squares sense by
 *   q(u, v) = a + b u + c v + d u^2 + e v^2 + f u v,  u, v in {-1, 0, 1};
 * the stationary point of q gives the offset (u*, v*) and q(u*, v*) the
 * refined response, H = [[2d, f], [f, 2e]] is the Hessian of Eq. 9, and the
 * keypoint is kept when H is negative definite, Tr(H)^2 / Det(H) <
 * (r+1)^2 / r (Eq. 12, r = edge_ratio) and |u*|, |v*| <= 1.
 *   det       (device) N x H x W detector responses (kaze_detector_response).
 *   kps       (device) extrema as written by kaze_find_extrema; an entry
 *             without a full 3x3 window in its level gets kept = 0 and NaN
 *             response and edge_ratio.
 *   count     (device) 1 int: the number of extrema (read on the device).
 *   capacity  entries of kps and out.
 *   edge_ratio  r of Eq. 12, > 1 (the paper gives none; 10 is SIFT's).
 *   out       (device) capacity entries; entry i refines kps[i].
 */
kaze_status kaze_refine_keypoints(const float* det, int W, int H, const kaze_params* p,
                                  const kaze_keypoint* kps, const int* count, int capacity,
                                  double edge_ratio, kaze_keypoint_refined* out,
                                  void* stream);

/*
 * Description stage (Sec. II-C, Sec. III-C).
 *
 * kaze_derivatives: scale-normalised first derivatives of every level,
 *   Lx = sigma_n D_x L and Ly = sigma_n D_y L, with the concatenated Scharr
 *   filter of Eq. 8 (step round(sigma_n), reflected border).
 *   levels   (device) N x H x W float32 input.
 *   lx, ly   (device) N x H x W float32 outputs (distinct from levels).
 */
kaze_status kaze_derivatives(const float* levels, int W, int H, const kaze_params* p,
                             float* lx, float* ly, void* stream);

/*
 * kaze_describe_keypoints: dominant orientation and 64-D M-SURF descriptor
 * of keypoint i < min(*count, capacity), at its (sub-pixel) position, with
 * the scale unit s = sigma_i of its level (Eq. 6).  Samples are bilinear in
 * Lx and Ly (pixel centres at integers, reflected outside the image).
 *   Orientation: responses w (Lx, Ly) at (x, y) + s (u, v) for integers
 *   u^2 + v^2 <= 36, w = exp(-(u^2 + v^2) / 12.5); the angle of the longest
 *   sum over a sliding pi/3 sector.
 *   Descriptor: 4 x 4 subregions of 9 x 9 samples of step s centred at
 *   -7.5, -2.5, 2.5, 7.5 s along and across the orientation; sums of the
 *   turned derivatives and their magnitudes weighted by a Gaussian of 2.5 s
 *   at the subregion centre, and per subregion by a Gaussian of 1.5
 *   subregions over the 4 x 4 mask; unit length.  Order: subregion row
 *   (across), column (along), then (sum d_u, sum d_v, sum |d_u|, sum |d_v|).
 *   lx, ly       (device) from kaze_derivatives.
 *   kps, count   (device) as written by kaze_refine_keypoints and
 *                kaze_find_extrema; entries with a level outside [0, N) or a
 *                non-finite position get angle NaN and a zero descriptor.
 *   angles       (device) capacity floats (radians, atan2 convention).
 *   descriptors  (device) capacity x 64 floats.
 */
kaze_status kaze_describe_keypoints(const float* lx, const float* ly, int W, int H,
                                    const kaze_params* p, const kaze_keypoint_refined* kps,
                                    const int* count, int capacity, float* angles,
                                    float* descriptors, void* stream);

/* Message for the most recent non-OK status returned on this thread. */
const char* kaze_last_error(void);

/*
 * Kernel timing hook for measurement.  kaze_profile_begin(names) makes every
 * following launch of the listed kernels (comma-separated names from
 * kaze_kernel_names()) record a pair of hipEvents around it on its stream,
 * up to 65536 launches.  kaze_profile_end() stops recording and reports,
 * after synchronising on the recorded events, the number of launches and
 * their summed duration in milliseconds.  Not thread safe.
 */
kaze_status kaze_profile_begin(const char* kernel_names);
kaze_status kaze_profile_end(int* launches, double* total_ms);

/* Comma-separated names of the library's kernels. */
const char* kaze_kernel_names(void);

/*
 * Streaming copy of n floats (device to device) with the library's own
 * vector-load kernel: a measurement of attainable HBM bandwidth and a
 * reference point for hardware byte counters.
 */
kaze_status kaze_copy_f32(const float* src, float* dst, size_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KAZE_H */
