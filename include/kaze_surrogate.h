/*
 * kaze_surrogate.h - C ABI of the learned surrogate for one AOS step of the
 * KAZE nonlinear scale space (libkaze, MI355X / gfx950).
 *
 * The scale space of Sec. II-A advances every level by one semi-implicit
 * step (Eq. 4).  The surrogate approximates that step with a residual
 * network, L_next ~ L + f(L, g, tau), where L is the previous level, g its
 * conductivity (Eqs. 2-3) and tau the step size.  The paper names learned
 * diffusion only as related work (trainable nonlinear reaction diffusion,
 * Sec. V); the network here is this library's own definition:
 *
 *   input planes (L, g, tau / 68), six 3x3 convolutions (cross-correlation,
 *   one pixel of zero padding) 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 with a
 *   bias per output channel and ReLU after layers 1..5; f is the output of
 *   layer 6 divided by 64 (a fixed scale: one step moves a level by about
 *   1e-3 while the hidden activations are of order one).  Loss: mean over
 *   all pixels of w_s (f - (L_next - L))^2, w_s a weight per sample.
 *
 * Parameters are one flat FP32 vector of kaze_sg_param_count() = 38,177
 * values: for each layer the weights [co][ci][3][3], then the biases [co].
 *
 * Arithmetic: BF16 MFMA operands with FP32 accumulation.  Layer 1 takes L, g
 * and its weights as three-term BF16 splits (about 16 significant bits); the
 * tau plane is applied in FP32.  Weights of layers 2..6 and the outputs of
 * layers 1..5 are BF16; f is FP32.  In the backward pass the gradient
 * entering each layer is stored in BF16; weight gradients are reduced in
 * FP32 in a fixed order (bitwise reproducible).
 *
 * Conventions are those of kaze.h: (device) pointers are HIP device
 * pointers, calls enqueue on `stream` and return without synchronising,
 * argument errors return synchronously, the caller owns every buffer
 * (the library allocates no device memory) and kaze_last_error() describes
 * the last failure.
 */
#ifndef KAZE_SURROGATE_H
#define KAZE_SURROGATE_H

#include <stddef.h>

#include "kaze.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP32 parameters of the network (38,177). */
int kaze_sg_param_count(void);

/* Bytes of the packed-weight buffer that kaze_sg_pack() writes. */
size_t kaze_sg_packed_bytes(void);

/*
 * Converts the flat FP32 parameters into the packed BF16 / FP32 operand
 * layout that the kernels read.  Must be called again after every change of
 * the parameters.
 *   params   (device) kaze_sg_param_count() floats.
 *   packed   (device) kaze_sg_packed_bytes() bytes, 256-byte aligned.
 */
kaze_status kaze_sg_pack(const float* params, void* packed, void* stream);

/*
 * A plan fixes the batch geometry: n samples of W x H pixels (1 <= W, H <=
 * 8192, 1 <= n <= 4096), for inference only (training = 0) or for forward
 * and backward passes (training = 1).  Its workspace holds the activations
 * and must not be used for anything else while the plan exists.
 */
typedef struct kaze_sg_plan kaze_sg_plan;

/* Workspace bytes for a plan, or 0 for invalid arguments. */
size_t kaze_sg_workspace_bytes(int n, int W, int H, int training);

/*
 * Creates a plan over the workspace `ws` (device, 256-byte aligned, at least
 * kaze_sg_workspace_bytes() bytes) and enqueues its zero fill on `stream`.
 * *out receives a host object released by kaze_sg_plan_destroy().
 */
kaze_status kaze_sg_plan_create(int n, int W, int H, int training, void* ws, size_t ws_bytes,
                                void* stream, kaze_sg_plan** out);
void kaze_sg_plan_destroy(kaze_sg_plan* plan);

/*
 * Forward pass over the plan's n samples.
 *   packed   (device) output of kaze_sg_pack().
 *   L, g     (device) n x H x W float32 each: previous level, conductivity.
 *   tau      (device) n float32 step sizes.
 *   out      (device) n x H x W float32: L + f if add_input, else f.  It
 *            may alias L or g (both are consumed before out is written).
 * Calls that share a plan must be ordered on one stream.
 */
kaze_status kaze_sg_forward(const kaze_sg_plan* plan, const void* packed, const float* L,
                            const float* g, const float* tau, float* out, int add_input,
                            void* stream);

/*
 * Forward and backward pass of the residual loss over the plan's n samples
 * (training plan only).
 *   L_next   (device) n x H x W float32 target levels.
 *   weight   (device) n float32 loss weights, or NULL for weight 1.
 *   grad     (device) output, kaze_sg_param_count() floats: d loss / d params
 *            (straight-through for the BF16 rounding of the weights).
 *   loss     (device) output, 1 float: mean over the n H W pixels of
 *            w_s (f - (L_next - L))^2.
 */
kaze_status kaze_sg_gradients(const kaze_sg_plan* plan, const void* packed, const float* L,
                              const float* g, const float* tau, const float* L_next,
                              const float* weight, float* grad, float* loss, void* stream);

/*
 * One Adam update (Kingma and Ba, with bias correction) of `count` FP32
 * parameters in place; m and v are the moment buffers (zero before step 1),
 * step counts from 1.
 */
kaze_status kaze_sg_adam(float* params, const float* grad, float* m, float* v, int count,
                         int step, double lr, double beta1, double beta2, double eps,
                         void* stream);


/*
 * Surrogate scale space: the scale space of kaze_build_scale_space() in
 * which the step into every level i >= 1 is first taken by the surrogate,
 * L_i = L_{i-1} + f(L_{i-1}, g, tau_i), and checked on probe windows: on
 * each window the exact AOS step of Eq. 4 is computed (every row and column
 * through the window solved whole) and compared with the surrogate's
 * result.  The level keeps the surrogate step iff the largest absolute
 * difference over its windows is <= bound; otherwise the step is recomputed
 * by AOS exactly as kaze_build_scale_space() does.  The decision is taken
 * on the device; nothing is copied to the host.
 */
typedef struct {
    double bound;     /* accept a level iff its probe error <= bound; a negative
                         bound always falls back, +inf never does           */
    int probes;       /* probe windows per level, 0..16 (0: no check, the
                         bound alone decides: accept iff bound >= 0)        */
    int probe_size;   /* edge of a probe window, 8..32 (clipped at the border) */
    int aos_shape;    /* tile shape of the AOS steps (values of
                         kaze_batch_config.aos_shape; -1 = 0)               */
} kaze_sg_config;

/* Defaults: bound 6.6e-5 per level, 4 probes of 32 x 32, AOS tile shape 0.
 * The bound is the surrogate's error budget of 1e-3 over the 15 steps of the
 * default schedule spread evenly: with the conductivity held fixed an AOS
 * step does not amplify a perturbation of its input in the maximum norm
 * (its matrix has a non-negative inverse with unit row sums), so the errors
 * of the accepted steps add up to at most 15 x 6.6e-5 = 9.9e-4 to first
 * order. */
kaze_status kaze_sg_default_config(kaze_sg_config* c);

typedef struct kaze_sg_scale_space kaze_sg_scale_space;

/* Workspace bytes for one W x H image, or 0 if the arguments are invalid. */
size_t kaze_sg_scale_space_workspace_bytes(int W, int H, const kaze_params* p,
                                           const kaze_sg_config* c);

/*
 * Prepares the surrogate scale space of one image and captures its launch
 * sequence.  The buffers are bound at creation; each run recomputes them.
 *   image    (host) one kaze_image_desc (kaze.h): img, levels, k are required;
 *            det and count (with kps/capacity) optional as for batches.
 *   packed   (device) output of kaze_sg_pack(); read by every run.
 *   probe_xy (host) N x probes x 2 ints: top-left corner (x, y) of each probe
 *            window of level i at [(i * probes + q) * 2]; level 0 is unused.
 *            Read during the call only; may be NULL when probes = 0.
 *   err      (device) N floats written by every run: err[i] = largest
 *            absolute difference between the surrogate and the exact step
 *            on level i's windows (0 with no probes; +inf for a non-finite
 *            result); err[0] = 0.  Level i used the surrogate iff
 *            err[i] <= bound.
 *   ws       (device) kaze_sg_scale_space_workspace_bytes() bytes, 256-byte
 *            aligned, owned by the object until it is destroyed.
 */
kaze_status kaze_sg_scale_space_create(const kaze_image_desc* image, const kaze_params* p,
                                       const kaze_sg_config* c, const void* packed,
                                       const int* probe_xy, float* err, void* ws,
                                       size_t ws_bytes, kaze_sg_scale_space** out);

/* Runs the whole sequence on `stream`: replays the captured graphs, or
 * enqueues the launches one by one if eager.  Runs of one object must be
 * ordered on one stream. */
kaze_status kaze_sg_scale_space_run(kaze_sg_scale_space* s, int eager, void* stream);

kaze_status kaze_sg_scale_space_destroy(kaze_sg_scale_space* s);

/*
 * Surrogate batches: the surrogate scale space above for many images of
 * different sizes in one plan.  Every phase of a level is one launch over
 * all images: the conductivity, the network input, the network and the
 * exact solves on every image's probe windows, the network on every image
 * whose level was accepted and the AOS step of Eq. 4 on every image whose
 * level was rejected, each decided per image and level on the device.  Base
 * image, contrast factor, detector response and extrema are those of
 * kaze_batch_create (kaze.h); the detector runs after the steps.
 *
 * The plan is a kaze_batch: kaze_batch_run, kaze_batch_properties and
 * kaze_batch_destroy apply to it.
 *   images    (host) n kaze_image_desc, as for kaze_batch_create.
 *   c         probe check and AOS tile shape (c->aos_shape, -1 = 0).
 *   packed    (device) output of kaze_sg_pack(); read by every run.
 *   probe_xy  (host) n x N x probes x 2 ints: top-left corner (x, y) of
 *             probe window q of image j, level i, at
 *             [((j * N + i) * probes + q) * 2]; level 0 is unused; may be
 *             NULL when probes = 0.
 *   err       (device) n x N floats written by every run: err[j * N + i] is
 *             the probe error of image j, level i (as for one image); image
 *             j used the surrogate for level i iff err[j * N + i] <= bound.
 *   ws        (device) kaze_sg_batch_workspace_bytes() bytes, 256-byte
 *             aligned, owned by the plan until it is destroyed.
 * Limits: n <= 4096; p->scheme AOS and p->substeps 1.
 */
size_t kaze_sg_batch_workspace_bytes(const kaze_image_desc* images, int n,
                                     const kaze_params* p, const kaze_sg_config* c);

kaze_status kaze_sg_batch_create(const kaze_image_desc* images, int n, const kaze_params* p,
                                 const kaze_sg_config* c, const void* packed,
                                 const int* probe_xy, float* err, void* ws, size_t ws_bytes,
                                 kaze_batch** out);

#ifdef __cplusplus
}
#endif

#endif /* KAZE_SURROGATE_H */
