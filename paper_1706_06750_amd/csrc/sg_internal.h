// Internal declarations of the learned surrogate for one AOS step: a
// residual stack of six 3x3 convolutions (3 -> 32 x5 -> 1) evaluated with
// BF16 MFMA implicit GEMMs that accumulate in FP32.
//
// Data layouts (all device memory, BF16 unless stated):
//   NHWC padded : [n][H+2][W+2][C], a one-pixel zero ring around every
//                 sample; pixel (y, x) at row y+1, column x+1.  Inputs of the
//                 forward and input-gradient convolutions (C = 8 or 32).
//   planar X    : [n][H+2][C][PX], same ring, one row of one channel
//                 contiguous; PX = 32 ceil(W/32) + 32.  Layer inputs for the
//                 weight gradient.
//   planar dZ   : [n][H][C][PZ], no ring, PZ = 32 ceil(W/32).  Gradients of
//                 the layer outputs for the weight gradient.
// Every ring and every column beyond W stays zero: the workspace is zero
// filled once when a plan is created and the kernels write interiors only.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace kaze {
namespace sg {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 6;
constexpr int kCh = 32;                 // hidden channels
constexpr float kTauRef = 68.0f;        // the tau input plane holds tau / kTauRef
constexpr float kOutScale = 1.0f / 64;  // f = kOutScale * (output of layer 6)
constexpr int kParams = (3 * 32 * 9 + 32) + 4 * (32 * 32 * 9 + 32) + (32 * 9 + 1);
constexpr int kPartStride = 9 * 32 * 32 + 32;  // weight-gradient partial of one wave
constexpr int kStrip = 16;              // output pixels per MFMA column block
constexpr int kWgStrip = 32;            // pixels per weight-gradient K block
constexpr int kConvRows = 32;           // output rows per wave of the convolutions
constexpr int kProbeHalo = 6;           // receptive-field radius of the six layers
constexpr int kPairOut = 112;           // output columns per block of a fused layer pair

// Offsets of layer l's weights and biases in the flat FP32 parameter vector
// (weights [co][ci][3][3], then biases [co]).
struct ParamLayout {
    int w[kLayers], b[kLayers], ci[kLayers], co[kLayers];
};
ParamLayout param_layout();

// Packed weights read by the kernels (one buffer, offsets in bytes).  A
// fragment is 64 lanes x 8 BF16 = the A operand of one 16x16x32 MFMA.
//   fwd[l]  : forward fragments of layer l, [MB][KS][64] x 8
//   dgr[l]  : input-gradient fragments of layer l (l >= 1), transposed and
//             flipped taps, [2][KS][64] x 8
//   bias[l] : FP32 [32] (zero beyond co)
//   tauw    : FP32 [32][9] layer-1 tap weights of the tau plane
struct PackLayout {
    size_t fwd[kLayers], dgr[kLayers], bias[kLayers], tauw, bytes;
};
PackLayout pack_layout();

struct Geo {
    int n, W, H;
    int strips;  // ceil(W / 16)
    int chunks;  // ceil(H / R)
    int R;       // output rows per wave
    int pw;      // padded row pitch in pixels (W + 2)
    long long sx;  // padded pixels per sample ((H + 2) (W + 2))
    int PX, PZ;    // planar pitches
};
Geo make_geo(int n, int W, int H, int R);

// Inference geometry of one image (the fields the forward kernels read).
__host__ __device__ inline Geo image_geo(int W, int H, int R) {
    Geo g;
    g.n = 1;
    g.W = W;
    g.H = H;
    g.R = R;
    g.strips = (W + kStrip - 1) / kStrip;
    g.chunks = (H + R - 1) / R;
    g.pw = W + 2;
    g.sx = (long long)(H + 2) * (W + 2);
    g.PX = g.PZ = 0;
    return g;
}

// One image of a batched forward launch (images of different sizes): its
// planes for the level being produced and the offset of its padded NHWC
// activations inside the batch's shared activation buffers.
struct SgImage {
    long long xoff;     // padded pixels of the images before it
    const float* L;     // previous level, [H][W]
    float* Lnext;       // the level produced: L + f
    const float* g;     // conductivity of L, [H][W]
    const float* gate;  // its probe error for this level (gated launches)
    int W, H;
};

// Work list of a batched launch: item t is (image, local item), the local
// item numbered as in the single-image launch of that image's geometry.
// imgs == NULL: a single-image launch over the Geo passed with it.
struct SgWork {
    const SgImage* imgs;
    const int2* items;
    int count;
};

enum Epi { EPI_RELU = 0, EPI_MASK = 1, EPI_OUT = 2 };

struct ConvArgs {
    const bf16* in;       // NHWC padded input, CIN channels
    const bf16x8* wfrag;  // packed fragments
    const float* bias;    // FP32 [16 MB] (EPI_RELU, EPI_OUT)
    const float* tauw;    // layer 1: FP32 [32][9] tau tap weights, else NULL
    const float* tau;     // [n] step sizes (layer 1)
    bf16* out;            // NHWC padded output, 32 channels (EPI_RELU, EPI_MASK)
    bf16* outp;           // planar copy of the output (X or dZ layout), or NULL
    const bf16* mask;     // EPI_MASK: NHWC padded activations of the layer below
    float* fout;          // EPI_OUT: [n][H][W] FP32
    const float* base;    // EPI_OUT: added to f (residual), or NULL
    const int* items;     // optional list of (chunk * strips + strip) of sample 0
    int nitems;
    const float* gate;    // optional: the launch runs only if *gate <= bound
    float bound;
    // batched inference (bw.imgs set): items, geometry and planes per image;
    // in, out index the shared activation buffers at each image's offset,
    // fout and base are the image's Lnext and L; with gate non-NULL every
    // image runs only if its own SgImage::gate holds a value <= bound
    SgWork bw;
};

hipError_t launch_conv(int cin, int mb, int epi, bool tau_term, const ConvArgs& a,
                       const Geo& g, hipStream_t s);

// Two consecutive layers in one pass (inference, whole image): layer a
// CINA -> 32 with ReLU (CINA = 8: layer 1 with the tau plane), then layer b
// 32 -> 32 with ReLU (MBB = 2) or 32 -> 1 output (MBB = 1).  Layer a's
// output stays on chip; results equal two conv_kernel launches bitwise.
struct Conv2Args {
    const bf16* in;       // NHWC padded input of layer a, CINA channels
    const bf16x8* wa;     // layer a fragments [2][KSA][64]
    const float* ba;      // layer a bias [32]
    const float* tauw;    // layer 1: FP32 [32][9] tau tap weights
    const float* tau;     // layer 1: step sizes [n]
    const bf16x8* wb;     // layer b fragments [MBB][9][64]
    const float* bb;      // layer b bias [32]
    bf16* out;            // MBB == 2: NHWC padded output, 32 channels
    float* fout;          // MBB == 1: [n][H][W] output
    const float* base;    // MBB == 1: added to f, or NULL
    const float* gate;    // optional: run only if *gate <= bound
    float bound;
    SgWork bw;            // batched inference, as in ConvArgs
};

hipError_t launch_conv2(int cina, int mbb, const Conv2Args& a, const Geo& g, hipStream_t s);
hipError_t launch_pack_input(const float* L, const float* gc, const float* tau, bf16* x0,
                             bf16* x0p, const Geo& g, hipStream_t s);
// Layer-1 input of every image of a batch (L and g of its SgImage entry)
// into the shared NHWC8 buffer x0 at the image's offset.
hipError_t launch_pack_input_batch(const SgImage* imgs, int n, bf16* x0, hipStream_t s);
hipError_t launch_loss(const float* f, const float* L, const float* Ln, const float* wts, bf16* dz6,
                       bf16* dz6p, float* lpart, int nblocks, const Geo& g, hipStream_t s);
int loss_blocks(const Geo& g);
hipError_t launch_wgrad(int cin, int cout, const bf16* xp, const bf16* dzp, float* part,
                        const Geo& g, int R, hipStream_t s);
int wgrad_items(const Geo& g, int R);
hipError_t launch_wreduce(int layer, const float* part, int items, float* grad, hipStream_t s);
hipError_t launch_sum(const float* v, int count, float scale, float* out, hipStream_t s);
hipError_t launch_pack_weights(const float* params, void* packed, hipStream_t s);
hipError_t launch_adam(float* p, const float* grad, float* m, float* v, int count, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace sg
}  // namespace kaze
