// C ABI of the learned AOS-step surrogate: argument checks, workspace layout
// and the launch sequences of the forward pass, the backward pass and Adam.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdlib.h>

#include "kaze.h"
#include "kaze_surrogate.h"
#include "sg_internal.h"

namespace kaze {
kaze_status set_error(kaze_status st, const char* fmt, va_list ap);
}

using namespace kaze::sg;

struct kaze_sg_plan {
    int n, W, H, training;
    Geo g;
    int wg_rows, wg_items, loss_blocks;
    // NHWC padded activations: x[0] has 8 channels, x[1..5] 32
    bf16* x[6];
    // planar copies of the layer inputs (training)
    bf16* xp[6];
    // gradients entering each layer: NHWC padded (dz[5]: 8 channels) and planar
    bf16* dz[6];
    bf16* dzp[6];
    float* f;
    float* part;
    float* lpart;
};

namespace {

constexpr int kWgRows = 64;    // rows per wave of the weight gradient

kaze_status fail(kaze_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    kaze::set_error(st, fmt, ap);
    va_end(ap);
    return st;
}

#define SG_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(KAZE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool dims_ok(int n, int W, int H) {
    return n >= 1 && n <= 4096 && W >= 1 && W <= 8192 && H >= 1 && H <= 8192;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace regions in order; with base == 0 only the total is computed.
size_t layout(int n, int W, int H, int training, uintptr_t base, kaze_sg_plan* p) {
    const Geo g = make_geo(n, W, H, kConvRows);
    const size_t nhwc = (size_t)n * g.sx;  // padded pixels
    const size_t planx = (size_t)n * (H + 2) * g.PX;
    const size_t planz = (size_t)n * H * g.PZ;
    const int wg_items = wgrad_items(g, kWgRows);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return (void*)(base ? base + at : 0);
    };
    bf16* x[6];
    x[0] = (bf16*)take(nhwc * 8 * 2);
    if (training) {
        for (int l = 1; l < 6; ++l) x[l] = (bf16*)take(nhwc * 32 * 2);
    } else {  // ping-pong pair
        x[1] = (bf16*)take(nhwc * 32 * 2);
        x[2] = (bf16*)take(nhwc * 32 * 2);
        for (int l = 3; l < 6; ++l) x[l] = x[1 + (l - 1) % 2];
    }
    bf16 *xp[6] = {}, *dz[6] = {}, *dzp[6] = {};
    float *f = nullptr, *part = nullptr, *lpart = nullptr;
    if (training) {
        xp[0] = (bf16*)take(planx * 8 * 2);
        for (int l = 1; l < 6; ++l) xp[l] = (bf16*)take(planx * 32 * 2);
        f = (float*)take((size_t)n * W * H * 4);
        dz[5] = (bf16*)take(nhwc * 8 * 2);
        for (int l = 1; l < 5; ++l) dz[l] = (bf16*)take(nhwc * 32 * 2);
        dzp[5] = (bf16*)take(planz * 1 * 2);
        for (int l = 0; l < 5; ++l) dzp[l] = (bf16*)take(planz * 32 * 2);
        part = (float*)take((size_t)wg_items * kPartStride * 4);
        lpart = (float*)take(1024 * 4);
    }
    if (p) {
        p->n = n;
        p->W = W;
        p->H = H;
        p->training = training;
        p->g = g;
        p->wg_rows = kWgRows;
        p->wg_items = wg_items;
        p->loss_blocks = loss_blocks(g);
        for (int l = 0; l < 6; ++l) {
            p->x[l] = x[l];
            p->xp[l] = xp[l];
            p->dz[l] = dz[l];
            p->dzp[l] = dzp[l];
        }
        p->f = f;
        p->part = part;
        p->lpart = lpart;
    }
    return o;
}

kaze_status check_plan(const kaze_sg_plan* p, const void* packed, const float* L, const float* g,
                       const float* tau) {
    if (!p) return fail(KAZE_ERR_INVALID_ARG, "plan is NULL");
    if (!packed || !L || !g || !tau) return fail(KAZE_ERR_INVALID_ARG, "NULL buffer");
    if (((uintptr_t)packed & 255) != 0)
        return fail(KAZE_ERR_INVALID_ARG, "packed weights must be 256-byte aligned");
    return KAZE_OK;
}

// Forward pass; with a training plan the planar copies are written too.
kaze_status forward(const kaze_sg_plan* p, const unsigned char* pk, const float* L, const float* gc,
                    const float* tau, float* fout, const float* base, hipStream_t s) {
    const PackLayout P = pack_layout();
    const Geo& g = p->g;
    SG_HIP(launch_pack_input(L, gc, tau, p->x[0], p->training ? p->xp[0] : nullptr, g, s));
    if (!p->training) {  // three fused pairs of layers
        for (int pr = 0; pr < 3; ++pr) {
            Conv2Args c = {};
            const int la = 2 * pr, lb = la + 1;
            c.in = p->x[pr];
            c.wa = reinterpret_cast<const bf16x8*>(pk + P.fwd[la]);
            c.ba = reinterpret_cast<const float*>(pk + P.bias[la]);
            c.wb = reinterpret_cast<const bf16x8*>(pk + P.fwd[lb]);
            c.bb = reinterpret_cast<const float*>(pk + P.bias[lb]);
            if (pr == 0) {
                c.tauw = reinterpret_cast<const float*>(pk + P.tauw);
                c.tau = tau;
            }
            if (pr < 2) {
                c.out = p->x[pr + 1];
            } else {
                c.fout = fout;
                c.base = base;
            }
            SG_HIP(launch_conv2(pr == 0 ? 8 : 32, pr < 2 ? 2 : 1, c, g, s));
        }
        return KAZE_OK;
    }
    for (int l = 0; l < kLayers; ++l) {
        ConvArgs a = {};
        a.in = p->x[l];
        a.wfrag = reinterpret_cast<const bf16x8*>(pk + P.fwd[l]);
        a.bias = reinterpret_cast<const float*>(pk + P.bias[l]);
        if (l == 0) {
            a.tauw = reinterpret_cast<const float*>(pk + P.tauw);
            a.tau = tau;
        }
        if (l < kLayers - 1) {
            a.out = p->x[l + 1];
            a.outp = p->training ? p->xp[l + 1] : nullptr;
            SG_HIP(launch_conv(l == 0 ? 8 : 32, 2, EPI_RELU, l == 0, a, g, s));
        } else {
            a.fout = fout;
            a.base = base;
            SG_HIP(launch_conv(32, 1, EPI_OUT, false, a, g, s));
        }
    }
    return KAZE_OK;
}

}  // namespace

extern "C" {

int kaze_sg_param_count(void) { return kParams; }

size_t kaze_sg_packed_bytes(void) { return pack_layout().bytes; }

kaze_status kaze_sg_pack(const float* params, void* packed, void* stream) {
    if (!params || !packed) return fail(KAZE_ERR_INVALID_ARG, "NULL buffer");
    if (((uintptr_t)packed & 255) != 0)
        return fail(KAZE_ERR_INVALID_ARG, "packed weights must be 256-byte aligned");
    SG_HIP(launch_pack_weights(params, packed, (hipStream_t)stream));
    return KAZE_OK;
}

size_t kaze_sg_workspace_bytes(int n, int W, int H, int training) {
    if (!dims_ok(n, W, H) || (training != 0 && training != 1)) return 0;
    return layout(n, W, H, training, 0, nullptr);
}

kaze_status kaze_sg_plan_create(int n, int W, int H, int training, void* ws, size_t ws_bytes,
                                void* stream, kaze_sg_plan** out) {
    if (!out) return fail(KAZE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!dims_ok(n, W, H))
        return fail(KAZE_ERR_UNSUPPORTED, "need 1 <= n <= 4096 and 1 <= W, H <= 8192");
    if (training != 0 && training != 1) return fail(KAZE_ERR_INVALID_ARG, "training must be 0 or 1");
    const size_t need = layout(n, W, H, training, 0, nullptr);
    if (!ws || ((uintptr_t)ws & 255) != 0)
        return fail(KAZE_ERR_WORKSPACE, "workspace missing or not 256-byte aligned");
    if (ws_bytes < need)
        return fail(KAZE_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    kaze_sg_plan* p = static_cast<kaze_sg_plan*>(calloc(1, sizeof(kaze_sg_plan)));
    if (!p) return fail(KAZE_ERR_INVALID_ARG, "out of host memory");
    layout(n, W, H, training, (uintptr_t)ws, p);
    const hipError_t e = launch_zero(ws, need, (hipStream_t)stream);
    if (e != hipSuccess) {
        free(p);
        return fail(KAZE_ERR_HIP, "workspace fill failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return KAZE_OK;
}

void kaze_sg_plan_destroy(kaze_sg_plan* plan) { free(plan); }

kaze_status kaze_sg_forward(const kaze_sg_plan* plan, const void* packed, const float* L,
                            const float* g, const float* tau, float* out, int add_input,
                            void* stream) {
    kaze_status st = check_plan(plan, packed, L, g, tau);
    if (st != KAZE_OK) return st;
    if (!out) return fail(KAZE_ERR_INVALID_ARG, "out is NULL");
    return forward(plan, static_cast<const unsigned char*>(packed), L, g, tau, out,
                   add_input ? L : nullptr, (hipStream_t)stream);
}

kaze_status kaze_sg_gradients(const kaze_sg_plan* plan, const void* packed, const float* L,
                              const float* g, const float* tau, const float* L_next,
                              const float* weight, float* grad, float* loss, void* stream) {
    kaze_status st = check_plan(plan, packed, L, g, tau);
    if (st != KAZE_OK) return st;
    if (!plan->training) return fail(KAZE_ERR_INVALID_ARG, "plan was created for inference only");
    if (!L_next || !grad || !loss) return fail(KAZE_ERR_INVALID_ARG, "NULL buffer");
    const hipStream_t s = (hipStream_t)stream;
    const unsigned char* pk = static_cast<const unsigned char*>(packed);
    const PackLayout P = pack_layout();
    const Geo& gg = plan->g;
    st = forward(plan, pk, L, g, tau, plan->f, nullptr, s);
    if (st != KAZE_OK) return st;
    SG_HIP(launch_loss(plan->f, L, L_next, weight, plan->dz[5], plan->dzp[5], plan->lpart,
                       plan->loss_blocks, gg, s));
    SG_HIP(launch_sum(plan->lpart, plan->loss_blocks, (float)(1.0 / ((double)gg.n * gg.W * gg.H)),
                      loss, s));
    // layer index l = 5 .. 0: weight gradient from (input of l, dZ of l), then
    // the input gradient masked by the ReLU of layer l-1
    for (int l = kLayers - 1; l >= 0; --l) {
        const int cin = l == 0 ? 8 : 32, cout = l == kLayers - 1 ? 1 : 32;
        SG_HIP(launch_wgrad(cin, cout, plan->xp[l], plan->dzp[l], plan->part, gg, plan->wg_rows, s));
        SG_HIP(launch_wreduce(l, plan->part, plan->wg_items, grad, s));
        if (l == 0) break;
        ConvArgs a = {};
        a.in = plan->dz[l];
        a.wfrag = reinterpret_cast<const bf16x8*>(pk + P.dgr[l]);
        a.mask = plan->x[l];
        a.out = l - 1 >= 1 ? plan->dz[l - 1] : nullptr;
        a.outp = plan->dzp[l - 1];
        SG_HIP(launch_conv(l == kLayers - 1 ? 8 : 32, 2, EPI_MASK, false, a, gg, s));
    }
    return KAZE_OK;
}

kaze_status kaze_sg_adam(float* params, const float* grad, float* m, float* v, int count, int step,
                         double lr, double beta1, double beta2, double eps, void* stream) {
    if (!params || !grad || !m || !v) return fail(KAZE_ERR_INVALID_ARG, "NULL buffer");
    if (count < 1 || step < 1) return fail(KAZE_ERR_INVALID_ARG, "count and step must be >= 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(KAZE_ERR_INVALID_ARG, "invalid Adam hyper-parameters");
    const double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
    SG_HIP(launch_adam(params, grad, m, v, count, (float)lr, (float)beta1, (float)beta2, (float)eps,
                       (float)c1, (float)c2, (hipStream_t)stream));
    return KAZE_OK;
}

}  // extern "C"
