// Host side of the learned-guess network: workspace layout, parameter handling,
// forward and backward passes of the BF16 U-Net and the Adam optimiser.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "net_internal.h"
#include "net_kernels.h"

using namespace mppnet;

namespace {

struct NetHipError {
  hipError_t e;
};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw NetHipError{e};
}

inline void ck_launch() { ck(hipGetLastError()); }

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

constexpr int kMaxParts = 512;      // weight-gradient partials per layer
constexpr int kMaxChanParts = 1024; // per-channel partials

bool shape_ok(int n, int bmax) { return n >= 16 && n <= 256 && n % 16 == 0 && bmax >= 1 && bmax <= 4096; }

size_t param_offsets(mpp_net_s* net) {
  size_t o = 0;
  for (int l = 0; l < kLayers; ++l) {
    net->off_w[l] = o;
    o += (size_t)27 * kSpec[l].co * kSpec[l].ci;
    net->off_b[l] = o;
    o += kSpec[l].co;
  }
  net->off_head = o;
  return o + kHeadCI + 1;
}

size_t net_layout(mpp_net_s* net, int n, int bmax, char* base) {
  Carver cv{base};
  net->n = n;
  net->bmax = bmax;
  net->nparams = param_offsets(net);
  const size_t P = net->nparams;
  net->w = cv.take<float>(P);
  net->g = cv.take<float>(P);
  net->m = cv.take<float>(P);
  net->v = cv.take<float>(P);
  for (int l = 0; l < kLayers; ++l) {
    net->wf[l] = cv.take<uint16_t>((size_t)kSpec[l].co * kpad(kSpec[l].cip));
    net->wb[l] = cv.take<uint16_t>((size_t)kSpec[l].cip * kpad(kSpec[l].co));
  }
  const size_t c0 = (size_t)n * n * n * bmax, c1 = c0 / 8, c2 = c0 / 64;
  const size_t cl[3] = {c0, c1, c2};
  net->x4 = cv.take<uint16_t>(c0 * 4);
  net->x8 = cv.take<uint16_t>(c0 * 8);
  for (int l = 0; l < kLayers; ++l) net->act[l] = cv.take<uint16_t>(cl[kSpec[l].level] * kSpec[l].co);
  net->p1 = cv.take<uint16_t>(c1 * 16);
  net->p2 = cv.take<uint16_t>(c2 * 32);
  net->g0a = cv.take<uint16_t>(c0 * 16);
  net->g0b = cv.take<uint16_t>(c0 * 16);
  net->g48 = cv.take<uint16_t>(c0 * 48);
  net->g1a = cv.take<uint16_t>(c1 * 32);
  net->g1b = cv.take<uint16_t>(c1 * 32);
  net->g96 = cv.take<uint16_t>(c1 * 96);
  net->gp1 = cv.take<uint16_t>(c1 * 16);
  net->g2a = cv.take<uint16_t>(c2 * 64);
  net->g2b = cv.take<uint16_t>(c2 * 64);
  net->gp2 = cv.take<uint16_t>(c2 * 32);
  size_t most = 0;
  for (int l = 0; l < kLayers; ++l) most = std::max(most, (size_t)kSpec[l].co * kpad(kSpec[l].cip));
  // a layer's partials: batch x chunks <= max(kMaxParts, batch) (conv_wgrad)
  net->part_floats = most * (size_t)std::max(kMaxParts, bmax);
  net->part = cv.take<float>(net->part_floats);
  net->cpart_floats = (size_t)kMaxChanParts * 64;
  net->cpart = cv.take<float>(net->cpart_floats);
  net->y = cv.take<float>(c0);
  net->tt = cv.take<float>(c0);
  net->dy = cv.take<float>(c0);
  net->lossb = cv.take<float>(bmax);
  net->coarse = cv.take<double>(c0 * 3);
  net->rms64 = cv.take<double>(bmax);
  net->rms32 = cv.take<float>(bmax);
  return cv.off + 256;
}

int level_n(const mpp_net_s* net, int level) { return net->n >> level; }

inline unsigned blocks(size_t work, int per) { return (unsigned)((work + per - 1) / per); }

// BF16 weight copies of the FP32 parameters
void prep_weights(mpp_net_s* net, hipStream_t s) {
  for (int l = 0; l < kLayers; ++l) {
    const LayerSpec& L = kSpec[l];
    const int kpf = kpad(L.cip), kpb = kpad(L.co);
    hipLaunchKernelGGL(k_prep_fwd, dim3(blocks((size_t)L.co * kpf, 256)), dim3(256), 0, s,
                       net->w + net->off_w[l], L.co, L.ci, L.cip, kpf, net->wf[l]);
    ck_launch();
    if (l > 0) {
      hipLaunchKernelGGL(k_prep_bwd, dim3(blocks((size_t)L.ci * kpb, 256)), dim3(256), 0, s,
                         net->w + net->off_w[l], L.co, L.ci, kpb, net->wb[l]);
      ck_launch();
    }
  }
  net->weights_fresh = true;
}

// the two sources of each layer's input
ConvSrc layer_src(const mpp_net_s* net, int l) {
  switch (l) {
    case 0: return ConvSrc{net->x8, nullptr, 0};
    case 2: return ConvSrc{net->p1, nullptr, 0};
    case 4: return ConvSrc{net->p2, nullptr, 0};
    case 6: return ConvSrc{net->act[5], net->act[3], 1};
    case 8: return ConvSrc{net->act[7], net->act[1], 1};
    default: return ConvSrc{net->act[l - 1], nullptr, 0};
  }
}

void conv_fwd(mpp_net_s* net, int l, int batch, hipStream_t s) {
  const int n = level_n(net, kSpec[l].level);
  const size_t cells = (size_t)n * n * n;
  const dim3 grid(blocks(cells, 16 * kConvMT * (kNetThreads / 64)), batch);
  const ConvSrc src = layer_src(net, l);
  const float* bias = net->w + net->off_b[l];
#define NET_FWD(CI, CA, CO)                                                                  \
  hipLaunchKernelGGL((k_conv<CI, CA, CO, 0>), grid, dim3(kNetThreads), 0, s, src, net->wf[l], \
                     bias, (const uint16_t*)nullptr, net->act[l], n)
  switch (l) {
    case 0: NET_FWD(8, 8, 16); break;
    case 1: NET_FWD(16, 16, 16); break;
    case 2: NET_FWD(16, 16, 32); break;
    case 3: NET_FWD(32, 32, 32); break;
    case 4: NET_FWD(32, 32, 64); break;
    case 5: NET_FWD(64, 64, 64); break;
    case 6: NET_FWD(96, 64, 32); break;
    case 7: NET_FWD(32, 32, 32); break;
    case 8: NET_FWD(48, 32, 16); break;
    case 9: NET_FWD(16, 16, 16); break;
  }
#undef NET_FWD
  ck_launch();
}

// data gradient of layer l: gradient gz of its pre-activation -> gradient of its input,
// times (mask > 0) when mask is given
void conv_dgrad(mpp_net_s* net, int l, const uint16_t* gz, const uint16_t* mask, uint16_t* out,
                int batch, hipStream_t s) {
  const int n = level_n(net, kSpec[l].level);
  const size_t cells = (size_t)n * n * n;
  const dim3 grid(blocks(cells, 16 * kConvMT * (kNetThreads / 64)), batch);
  const ConvSrc src{gz, nullptr, 0};
#define NET_DG(CI, CO)                                                                        \
  hipLaunchKernelGGL((k_conv<CI, CI, CO, 1>), grid, dim3(kNetThreads), 0, s, src, net->wb[l],  \
                     (const float*)nullptr, mask, out, n)
  switch (l) {
    case 1: NET_DG(16, 16); break;
    case 2: NET_DG(32, 16); break;
    case 3: NET_DG(32, 32); break;
    case 4: NET_DG(64, 32); break;
    case 5: NET_DG(64, 64); break;
    case 6: NET_DG(32, 96); break;
    case 7: NET_DG(32, 32); break;
    case 8: NET_DG(16, 48); break;
    case 9: NET_DG(16, 16); break;
    default: return;
  }
#undef NET_DG
  ck_launch();
}

// weight and bias gradients of layer l from the gradient gz of its pre-activation
void conv_wgrad(mpp_net_s* net, int l, const uint16_t* gz, int batch, hipStream_t s) {
  const LayerSpec& L = kSpec[l];
  const int n = level_n(net, L.level);
  const int cells = n * n * n;
  const int kp = kpad(L.cip);
  const int cols_per_block = 16 * kWgNT * (kNetThreads / 64);
  const int yblocks = (kp + cols_per_block - 1) / cols_per_block;
  // batch * chunks partials, at most max(kMaxParts, batch) (the buffer's size)
  int chunks = std::max(1, std::min(kMaxParts / batch, (2048 + batch * yblocks - 1) / (batch * yblocks)));
  int chunk_len = ((cells + chunks - 1) / chunks + 31) / 32 * 32;
  chunks = (cells + chunk_len - 1) / chunk_len;
  const int nparts = batch * chunks;
  // the partials must fit the buffer sized in net_layout (batches above kMaxParts once
  // overran it into the arrays after it)
  if ((size_t)nparts * L.co * kp > net->part_floats) throw NetHipError{hipErrorInvalidValue};
  const dim3 grid(nparts, yblocks);
  const ConvSrc src = layer_src(net, l);
#define NET_WG(CO, CI, CA)                                                                   \
  hipLaunchKernelGGL((k_wgrad<CO, CI, CA>), grid, dim3(kNetThreads), 0, s, src, gz, net->part, \
                     n, chunks, chunk_len)
  switch (l) {
    case 0: NET_WG(16, 8, 8); break;
    case 1: NET_WG(16, 16, 16); break;
    case 2: NET_WG(32, 16, 16); break;
    case 3: NET_WG(32, 32, 32); break;
    case 4: NET_WG(64, 32, 32); break;
    case 5: NET_WG(64, 64, 64); break;
    case 6: NET_WG(32, 96, 64); break;
    case 7: NET_WG(32, 32, 32); break;
    case 8: NET_WG(16, 48, 32); break;
    case 9: NET_WG(16, 16, 16); break;
  }
#undef NET_WG
  ck_launch();
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks((size_t)L.co * 27 * L.cip, 256)), dim3(256), 0,
                     s, net->part, nparts, L.co, kp, L.cip, L.ci, net->g + net->off_w[l]);
  ck_launch();
  // bias: channel sums of gz
  const size_t total = (size_t)cells * batch;
  const int per = (int)std::max<size_t>(4096, (total + kMaxChanParts - 1) / kMaxChanParts);
  const unsigned nb = blocks(total, per);
  hipLaunchKernelGGL(k_chan_sum, dim3(nb), dim3(kNetThreads), 0, s, gz, L.co, total, per,
                     net->cpart);
  ck_launch();
  hipLaunchKernelGGL(k_chan_reduce, dim3(1), dim3(64), 0, s, net->cpart, (int)nb, L.co,
                     net->g + net->off_b[l]);
  ck_launch();
}

void pool(const uint16_t* in, int C, int nc, int batch, uint16_t* out, hipStream_t s) {
  const size_t work = (size_t)nc * nc * nc * batch * (C / 8);
  hipLaunchKernelGGL(k_pool, dim3(blocks(work, 256)), dim3(256), 0, s, in, C, nc, batch, out);
  ck_launch();
}

void backward(mpp_net_s* net, const float* dy, int batch, hipStream_t s) {
  const int n = net->n;
  const size_t c0 = (size_t)n * n * n * batch;
  // head
  {
    const int per = (int)std::max<size_t>(4096, (c0 + kMaxChanParts - 1) / kMaxChanParts);
    const unsigned nb = blocks(c0, per);
    hipLaunchKernelGGL(k_head_bwd, dim3(nb), dim3(kNetThreads), 0, s, net->act[9],
                       net->w + net->off_head, dy, c0, per, net->g0a, net->cpart);
    ck_launch();
    hipLaunchKernelGGL(k_chan_reduce, dim3(1), dim3(64), 0, s, net->cpart, (int)nb, 17,
                       net->g + net->off_head);
    ck_launch();
  }
  const int n1 = n / 2, n2 = n / 4;
  // decoder, level 0
  conv_wgrad(net, 9, net->g0a, batch, s);
  conv_dgrad(net, 9, net->g0a, net->act[8], net->g0b, batch, s);
  conv_wgrad(net, 8, net->g0b, batch, s);
  conv_dgrad(net, 8, net->g0b, nullptr, net->g48, batch, s);
  {
    const size_t work = (size_t)n1 * n1 * n1 * batch * 32;
    hipLaunchKernelGGL(k_up_back, dim3(blocks(work, 256)), dim3(256), 0, s, net->g48, 48, 32, n1,
                       batch, net->act[7], net->g1a);
    ck_launch();
  }
  // decoder, level 1
  conv_wgrad(net, 7, net->g1a, batch, s);
  conv_dgrad(net, 7, net->g1a, net->act[6], net->g1b, batch, s);
  conv_wgrad(net, 6, net->g1b, batch, s);
  conv_dgrad(net, 6, net->g1b, nullptr, net->g96, batch, s);
  {
    const size_t work = (size_t)n2 * n2 * n2 * batch * 64;
    hipLaunchKernelGGL(k_up_back, dim3(blocks(work, 256)), dim3(256), 0, s, net->g96, 96, 64, n2,
                       batch, net->act[5], net->g2a);
    ck_launch();
  }
  // bottleneck
  conv_wgrad(net, 5, net->g2a, batch, s);
  conv_dgrad(net, 5, net->g2a, net->act[4], net->g2b, batch, s);
  conv_wgrad(net, 4, net->g2b, batch, s);
  conv_dgrad(net, 4, net->g2b, nullptr, net->gp2, batch, s);
  {
    const size_t work = (size_t)n1 * n1 * n1 * batch * 32;
    hipLaunchKernelGGL(k_skip_pool_back, dim3(blocks(work, 256)), dim3(256), 0, s, net->g96, 96,
                       64, net->gp2, 32, n1, batch, net->act[3], net->g1a);
    ck_launch();
  }
  // encoder, level 1
  conv_wgrad(net, 3, net->g1a, batch, s);
  conv_dgrad(net, 3, net->g1a, net->act[2], net->g1b, batch, s);
  conv_wgrad(net, 2, net->g1b, batch, s);
  conv_dgrad(net, 2, net->g1b, nullptr, net->gp1, batch, s);
  {
    const size_t work = (size_t)n * n * n * batch * 16;
    hipLaunchKernelGGL(k_skip_pool_back, dim3(blocks(work, 256)), dim3(256), 0, s, net->g48, 48,
                       32, net->gp1, 16, n, batch, net->act[1], net->g0a);
    ck_launch();
  }
  // encoder, level 0
  conv_wgrad(net, 1, net->g0a, batch, s);
  conv_dgrad(net, 1, net->g0a, net->act[0], net->g0b, batch, s);
  conv_wgrad(net, 0, net->g0b, batch, s);
}

// He-normal weights (std sqrt(2 / fan_in)), zero biases, zero head.
// Normal deviates by Box-Muller over a splitmix64 stream.
void init_params(mpp_net_s* net, uint64_t seed, std::vector<float>& h) {
  h.assign(net->nparams, 0.f);
  uint64_t state = seed;
  auto next = [&]() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto uniform = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  auto normal = [&]() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  };
  for (int l = 0; l < kLayers; ++l) {
    const double sd = std::sqrt(2.0 / (27.0 * kSpec[l].ci));
    const size_t cnt = (size_t)27 * kSpec[l].co * kSpec[l].ci;
    for (size_t i = 0; i < cnt; ++i) h[net->off_w[l] + i] = (float)(sd * normal());
  }
  // the head starts at zero: the first prediction is 0 (relative loss 1) instead of a
  // random field many times the target's size
}

int set_params_impl(mpp_net_s* net, const float* params, hipStream_t s) {
  const size_t bytes = sizeof(float) * net->nparams;
  ck(hipMemcpyAsync(net->w, params, bytes, hipMemcpyHostToDevice, s));
  ck(hipMemsetAsync(net->m, 0, bytes, s));
  ck(hipMemsetAsync(net->v, 0, bytes, s));
  ck(hipMemsetAsync(net->g, 0, bytes, s));
  ck(hipStreamSynchronize(s));
  net->step = 0;
  net->last_batch = 0;
  net->weights_fresh = false;
  return MPP_OK;
}

void forward_impl(mpp_net_s* net, const uint16_t* x4, float* y, int batch, hipStream_t s);

bool adam_args_ok(float lr, float beta1, float beta2, float eps) {
  return lr > 0.f && std::isfinite(lr) && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f &&
         beta2 < 1.f && eps > 0.f && std::isfinite(eps);
}

// One Adam step with the current gradient (bias corrections from the step count).
void adam_impl(mpp_net_s* net, float lr, float beta1, float beta2, float eps, hipStream_t s) {
  net->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, net->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, net->step)));
  hipLaunchKernelGGL(k_adam, dim3(blocks(net->nparams, 256)), dim3(256), 0, s, net->w, net->m,
                     net->v, net->g, net->nparams, lr, beta1, beta2, eps, c1, c2);
  ck_launch();
  net->weights_fresh = false;
}

}  // namespace

namespace mppnet {

int forward(mpp_net_s* net, const uint16_t* x4, float* y, int batch, hipStream_t s) {
  try {
    forward_impl(net, x4, y, batch, s);
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

}  // namespace mppnet

namespace {

void forward_impl(mpp_net_s* net, const uint16_t* x4, float* y, int batch, hipStream_t s) {
  const int n = net->n, n1 = n / 2, n2 = n / 4;
  const size_t c0 = (size_t)n * n * n * batch;
  if (!net->weights_fresh) prep_weights(net, s);
  hipLaunchKernelGGL(k_pad_input, dim3(blocks(c0, 256)), dim3(256), 0, s, x4, net->x8, c0);
  ck_launch();
  conv_fwd(net, 0, batch, s);
  conv_fwd(net, 1, batch, s);
  pool(net->act[1], 16, n1, batch, net->p1, s);
  conv_fwd(net, 2, batch, s);
  conv_fwd(net, 3, batch, s);
  pool(net->act[3], 32, n2, batch, net->p2, s);
  for (int l = 4; l < kLayers; ++l) conv_fwd(net, l, batch, s);
  hipLaunchKernelGGL(k_head_fwd, dim3(blocks(c0, 256)), dim3(256), 0, s, net->act[9],
                     net->w + net->off_head, c0, y);
  ck_launch();
  net->last_batch = batch;
}

}  // namespace

extern "C" {

int32_t mpp_net_param_count(void) {
  mpp_net_s tmp;
  return (int32_t)param_offsets(&tmp);
}

size_t mpp_net_workspace_bytes(int32_t n, int32_t batch_max) {
  if (!shape_ok(n, batch_max)) return 0;
  mpp_net_s tmp;
  return net_layout(&tmp, n, batch_max, nullptr);
}

int mpp_net_create(int32_t n, int32_t batch_max, uint64_t seed, void* workspace,
                   size_t workspace_bytes, void* stream, mpp_net* out) {
  if (out) *out = nullptr;
  if (!shape_ok(n, batch_max) || !workspace || !out) return MPP_EINVAL;
  mpp_net_s tmp;
  if (workspace_bytes < net_layout(&tmp, n, batch_max, nullptr)) return MPP_ENOMEM;
  mpp_net_s* net = new (std::nothrow) mpp_net_s();
  if (!net) return MPP_ENOMEM;
  char* base =
      reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(workspace) + 255) & ~uintptr_t(255));
  net_layout(net, n, batch_max, base);
  std::vector<float> h;
  init_params(net, seed, h);
  try {
    set_params_impl(net, h.data(), reinterpret_cast<hipStream_t>(stream));
  } catch (NetHipError&) {
    delete net;
    return MPP_EDEVICE;
  }
  *out = net;
  return MPP_OK;
}

void mpp_net_destroy(mpp_net net) { delete net; }

int mpp_net_set_params(mpp_net net, const float* params, void* stream) {
  if (!net || !params) return MPP_EINVAL;
  for (size_t i = 0; i < net->nparams; ++i)
    if (!std::isfinite(params[i])) return MPP_EINVAL;
  try {
    return set_params_impl(net, params, reinterpret_cast<hipStream_t>(stream));
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
}

int mpp_net_get_params(mpp_net net, float* params, void* stream) {
  if (!net || !params) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  try {
    ck(hipMemcpyAsync(params, net->w, sizeof(float) * net->nparams, hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

int mpp_net_get_grads(mpp_net net, float* grads, void* stream) {
  if (!net || !grads) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  try {
    ck(hipMemcpyAsync(grads, net->g, sizeof(float) * net->nparams, hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

int mpp_net_forward(mpp_net net, const uint16_t* x, float* y, int32_t batch, void* stream) {
  if (!net || !x || !y || batch < 1 || batch > net->bmax) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  try {
    const size_t c0 = (size_t)net->n * net->n * net->n * batch;
    if (x != net->x4)
      ck(hipMemcpyAsync(net->x4, x, c0 * 4 * sizeof(uint16_t), hipMemcpyDeviceToDevice, s));
    forward_impl(net, net->x4, y, batch, s);
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

int mpp_net_loss(mpp_net net, const float* y, const float* t, float* dy, float* loss,
                 int32_t batch, void* stream) {
  if (!net || !y || !t || !dy || !loss || batch < 1 || batch > net->bmax) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int cells = net->n * net->n * net->n;
  try {
    hipLaunchKernelGGL(k_loss, dim3(batch), dim3(1024), 0, s, y, t, cells, 1.0f / batch, dy, loss);
    ck_launch();
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

int mpp_net_backward(mpp_net net, const float* dy, int32_t batch, void* stream) {
  if (!net || !dy || batch < 1 || batch != net->last_batch) return MPP_EINVAL;
  try {
    backward(net, dy, batch, reinterpret_cast<hipStream_t>(stream));
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

int mpp_net_adam(mpp_net net, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!net || !adam_args_ok(lr, beta1, beta2, eps)) return MPP_EINVAL;
  try {
    adam_impl(net, lr, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream));
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

int mpp_net_train(mpp_net net, const uint16_t* x, const float* t, int64_t count,
                  const mpp_net_train_opts* o, float* losses, void* stream) {
  // everything that does not need the handle first (the handle is read last)
  if (!net || !x || !t || !o || count < 1 || o->batch < 1 || o->steps < 0 ||
      o->first_step < 0 || o->total_steps < 0 ||
      !adam_args_ok(o->lr0, o->beta1, o->beta2, o->eps) || !(o->lr1 > 0.f) ||
      !std::isfinite(o->lr1))
    return MPP_EINVAL;
  if (o->batch > net->bmax) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n = net->n, cells = n * n * n, B = o->batch;
  const unsigned gx = std::max(1u, std::min(blocks(cells, 256), 2048u / (unsigned)B));
  try {
    for (int32_t q = 0; q < o->steps; ++q) {
      const int64_t step = o->first_step + q;
      // learning rate of this step on the geometric schedule lr0 -> lr1 over total_steps
      double lr = o->lr0;
      if (o->total_steps > 1)
        lr = (double)o->lr0 * std::pow((double)o->lr1 / (double)o->lr0,
                                       (double)step / (double)(o->total_steps - 1));
      hipLaunchKernelGGL(k_gather_samples, dim3(gx, B), dim3(256), 0, s,
                         reinterpret_cast<const uint2*>(x), t, cells, (int64_t)count, o->seed,
                         step, B, reinterpret_cast<uint2*>(net->x4), net->tt);
      ck_launch();
      forward_impl(net, net->x4, net->y, B, s);
      float* lo = losses ? losses + (size_t)q * B : net->lossb;
      hipLaunchKernelGGL(k_loss, dim3(B), dim3(1024), 0, s, net->y, net->tt, cells, 1.0f / B,
                         net->dy, lo);
      ck_launch();
      backward(net, net->dy, B, s);
      adam_impl(net, (float)lr, o->beta1, o->beta2, o->eps, s);
    }
  } catch (NetHipError&) {
    return MPP_EDEVICE;
  }
  return MPP_OK;
}

}  // extern "C"
