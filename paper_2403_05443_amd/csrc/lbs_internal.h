// lbs_internal.h - the surrogate object behind the opaque lbs handle
// (internal; shared by the surrogate API and the warm start).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "lbell_launch.h"

struct lbs {
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    int max_n = 0, max_tiles = 0;
    long long adam_t = 0;  // Adam steps taken since the parameters were set
    // device regions
    float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr, *Lpart = nullptr, *gsum = nullptr;
    float *X = nullptr, *Y = nullptr, *out = nullptr;
    double* loss_acc = nullptr;
    std::string err;
};

namespace lbd {
// Layout of a surrogate arena for up to max_n samples (offsets in bytes).
struct LbsLayout {
    size_t P, M, V, G, Lpart, gsum, X, Y, out, loss, total;
};
LbsLayout lbs_layout(int max_n);
}  // namespace lbd
