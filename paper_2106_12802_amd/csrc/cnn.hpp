// Fusion-network internals shared by cnn.hip (kernels) and net.hip (host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "mrs.h"

namespace mrs {

enum ViewMode {
  VIEW_PLAIN = 0,             // NHWC tensor a with ca channels
  VIEW_CONCAT_UNSHUFFLE = 1,  // [a (ca ch, this res), unshuffle_r(b) (r^2 cb ch, from res*r)]
  VIEW_SHUFFLE_CONCAT = 2,    // [shuffle_r(a) (c0 ch, from res/r, ca = r^2 c0), b (cb ch)]
};

struct ConvArgs {
  int mode;
  const uint16_t* a;
  int ca;
  const uint16_t* b;
  int cb;
  int c0;
  int r;
  int B, H, W;  // output (and input) resolution of this conv
  int cin_p;    // channels per tap as laid out in K (multiple of 8)
  int taps;     // 1 or 9
  int kp;       // padded K (multiple of 32)
  const uint16_t* w;  // packed BF16 [cout_p][kp]
  const float* bias;  // [cout]
  int cout;
  int relu;
  const float* res;  // optional FP32 [M][cout]: y = res + res_scale * y
  float res_scale;
  const float* res2;  // optional FP32 [M][cout]: y += res2
  float* out_f;       // optional FP32 output, out_f_stride floats per pixel
  int out_f_stride;
  uint16_t* out_h;  // optional BF16 output, out_h_stride per pixel
  int out_h_stride;
};

struct NetLayer {
  const char* name;
  int cout, cin, k;
  int cin_p, kp, cout_p;
  int64_t w_off, b_off;  // offsets in the FP32 master vector
  int64_t pk_off;        // offset in the packed BF16 weights
};

constexpr int NET_FEAT = 64;
constexpr int NET_SCALE = 4;
constexpr int NET_NRES = 16;
constexpr int NET_UPCH = 16;
constexpr float NET_RES_SCALE = 0.1f;
constexpr int64_t NET_NUM_PARAMS = 1408883;

void launch_conv(const ConvArgs& a, int cout_p, hipStream_t st);
void launch_prep(int64_t nhr, int64_t nlr, const float* hr, const float* aux, const float* lr,
                 uint16_t* xh, uint16_t* xl, hipStream_t st);
void launch_pack(const float* wm, const NetLayer& L, uint16_t* wp, hipStream_t st);
void launch_init(float* dst, const NetLayer& L, uint64_t seed, hipStream_t st);

}  // namespace mrs

struct mrs_net {
  std::vector<mrs::NetLayer> layers;
  int64_t nparams = 0;
  int64_t npacked = 0;
  float* d_master = nullptr;
  uint16_t* d_packed = nullptr;
  bool has_params = false;
  // activation arena of the last forward (grown on demand)
  char* d_arena = nullptr;
  size_t arena_bytes = 0;
  // views of the last forward's activations (debug)
  int last_B = 0, last_H = 0, last_W = 0;
  float* last_f0 = nullptr;
  float* last_fdf = nullptr;
};
