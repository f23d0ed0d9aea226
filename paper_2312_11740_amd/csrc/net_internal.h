// Internal declarations of the learned-guess network shared by the solver's glue
// (features from an operator, the guess itself) and the network's own host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mpp.h"

namespace mppnet {

constexpr int kLayers = 10;     // 3x3x3 convolutions
constexpr int kHeadCI = 16;

// One convolution of the U-Net: real input channels ci (padded to cip, a multiple of
// 8), of which the first ca come from the first source; output channels co; the
// resolution level (0: n, 1: n/2, 2: n/4).
struct LayerSpec {
  int ci, cip, ca, co, level, up;
};

constexpr LayerSpec kSpec[kLayers] = {
    {4, 8, 8, 16, 0, 0},     // e1a
    {16, 16, 16, 16, 0, 0},  // e1b
    {16, 16, 16, 32, 1, 0},  // e2a (input: pooled e1)
    {32, 32, 32, 32, 1, 0},  // e2b
    {32, 32, 32, 64, 2, 0},  // b1 (input: pooled e2)
    {64, 64, 64, 64, 2, 0},  // b2
    {96, 96, 64, 32, 1, 1},  // d2a (input: up(b2) ++ e2b)
    {32, 32, 32, 32, 1, 0},  // d2b
    {48, 48, 32, 16, 0, 1},  // d1a (input: up(d2b) ++ e1b)
    {16, 16, 16, 16, 0, 0},  // d1b
};

}  // namespace mppnet

struct mpp_net_s {
  int n = 0, bmax = 0;
  size_t nparams = 0;
  size_t off_w[mppnet::kLayers] = {}, off_b[mppnet::kLayers] = {}, off_head = 0;
  int step = 0;            // Adam steps since creation / set_params
  int last_batch = 0;      // batch of the last forward (its activations are kept)
  bool weights_fresh = false;
  // FP32 parameters, gradient and Adam moments
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  // BF16 weights: forward [co][kpad(cip)] and data-gradient [cip][kpad(co)] layouts
  uint16_t* wf[mppnet::kLayers] = {};
  uint16_t* wb[mppnet::kLayers] = {};
  // activations (BF16, channels-last)
  uint16_t *x4 = nullptr, *x8 = nullptr;
  uint16_t* act[mppnet::kLayers] = {};
  uint16_t *p1 = nullptr, *p2 = nullptr;
  // gradients of the activations
  uint16_t *g0a = nullptr, *g0b = nullptr, *g48 = nullptr;
  uint16_t *g1a = nullptr, *g1b = nullptr, *g96 = nullptr, *gp1 = nullptr;
  uint16_t *g2a = nullptr, *g2b = nullptr, *gp2 = nullptr;
  float* part = nullptr;       // weight-gradient partials
  size_t part_floats = 0;
  float* cpart = nullptr;      // per-channel partials (bias and head gradients)
  size_t cpart_floats = 0;
  // scratch of the solver glue: network output, coarse means, rms per sample
  float* y = nullptr;          // [bmax][n^3]
  // training staging (mpp_net_train): targets of the drawn batch, dloss/dy, losses
  float* tt = nullptr;         // [bmax][n^3]
  float* dy = nullptr;         // [bmax][n^3]
  float* lossb = nullptr;      // [bmax]
  double* coarse = nullptr;    // [bmax][n^3][3]: mean 1/rho, mean b, mean p
  double* rms64 = nullptr;     // [bmax]
  float* rms32 = nullptr;      // [bmax]
};

namespace mppnet {

// y = net(x4) for `batch` samples on stream s (throws on HIP errors, as int codes)
int forward(mpp_net_s* net, const uint16_t* x4, float* y, int batch, hipStream_t s);

}  // namespace mppnet
