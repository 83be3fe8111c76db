// Parameter block of the learned bandwidth network and launcher declarations.
#pragma once

#include "internal.hpp"

namespace flp {

constexpr int kHidden = 64;
constexpr int kFeat = 5;
// float offsets in the parameter block: W1[64][5], b1[64], W2[64][64], b2[64],
// w3[64], b3, then the feature standardisation mu[5], sd[5]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kFeat;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;
constexpr int kTrain = kOffB3 + 1;          // 4609 trainable entries
constexpr int kOffMu = kTrain;
constexpr int kOffSd = kOffMu + kFeat;
constexpr int kParams = kOffSd + kFeat;     // 4619
constexpr float kSmax = 1.3862943611198906f; // ln 4

// up to four field planes, passed to kernels by value
struct Planes {
    const void* p[4];
};
struct MutPlanes {
    void* p[4];
};

template <typename R, int D>
// features (binary64) then the network (bf16 MFMA); cnt: 2 M words and zb:
// count 16-byte feature records of workspace
hipError_t launch_bandwidth_forward(const TrajDev& t, const MeshDev& m, const float* theta, unsigned int* cnt, void* zb,
                                    float* hfac, float* z, float* o, float* fraw, hipStream_t s);
template <typename R, int D>
hipError_t launch_traj_backward(const MeshDev& m, double cutoff, const uint32_t* keys, uint32_t sentinel,
                                const double4* rpos, const R* rw, Planes S, const void* den, Planes dLdS,
                                double scale, const void* cell_scale, float* bcells, float* eplane, float* out,
                                int64_t N, hipStream_t s);
int mlp_backward_blocks(int64_t N);
template <int D>
hipError_t launch_mlp_backward(const float* theta, int64_t N, const float* z, const float* o, const float* dlogh,
                               float* partial, int nblocks, float* grad, hipStream_t s);
// feature standardisation: moments over valid trajectories in a fixed order
constexpr int kMomParts = 1024 * 6;   // doubles of per-block partials
hipError_t launch_feat_moments(const float* fraw, int64_t N, int pass, const double* acc0, double* part, double* acc,
                               hipStream_t s);
hipError_t launch_feat_finish(const double* acc0, const double* acc1, float* theta, hipStream_t s);
hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int64_t step, double lr, double b1,
                       double b2, double eps, hipStream_t s);
template <typename R>
hipError_t launch_loss(int C, int64_t M, Planes S, Planes Rf, MutPlanes G, bool want_grad, double* part, double* res,
                       hipStream_t s);

}  // namespace flp
