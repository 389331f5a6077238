// Fast explicit diffusion (Eq. 5): declarations shared by the FED kernel and
// the host code.
#pragma once

#include <vector>

#include "kaze_internal.h"

namespace kaze {

// Stability limit of one explicit 5-point step with unit spacing and g <= 1.
constexpr double kFedTauMax = 0.25;
// Explicit steps per launch: a region of 64 x 64 pixels in LDS gives an
// output tile of (64 - 2 kFedS)^2 pixels after kFedS steps.  Measured at
// 1920x1200 (166 steps per image): 4 steps per launch 934 images/s, 6 996,
// 8 1100; the launches' fixed cost outweighs the wider recomputed ring.
constexpr int kFedS = 8;
constexpr int kFedRegion = 64;
constexpr int kFedTile = kFedRegion - 2 * kFedS;

// Step sizes of one cycle of total time T in application order (host,
// double; see kaze_fed_schedule in kaze.h).  Empty for T <= 0.
std::vector<double> fed_schedule(double T);

// The steps of one launch (at most kFedS), as multiples of the half flux
// sum: every step adds tau_j/2 * sum_q (g_p + g_q)(L_q - L_p).
struct FedSteps {
    int n;
    float half_tau[kFedS];
};

// One launch: up to kFedS explicit steps from src into dst (distinct
// buffers), conductivity g fixed; one image of W x H.
hipError_t launch_fed(const float* src, const float* g, float* dst, int W, int H,
                      const FedSteps& st, hipStream_t s);
inline int fed_tiles_of(int W, int H) {
    return ((W + kFedTile - 1) / kFedTile) * ((H + kFedTile - 1) / kFedTile);
}

}  // namespace kaze
