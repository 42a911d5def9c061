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

enum EpiMode { EPI_PLAIN = 0, EPI_REC_SPLIT = 1, EPI_FUSE_SPLIT = 2 };

// Epilogue of a data-gradient conv (output pixel m, channel n, value y).
struct BwdEpi {
  int mode;
  float scale;         // y *= scale first
  int stride;          // PLAIN: channels per pixel of add/mask/out; REC: of out_f;
                       // FUSE: channels of the HR tensor (h0)
  const float* add1;   // PLAIN: y += add1; FUSE (n >= c_split): y += add1[HR index]
  const float* add2;   // PLAIN: y += add2
  const uint16_t* mask;  // y = 0 where mask <= 0 (PLAIN; REC n < c_split; FUSE n < c_split)
  float* out_f;
  uint16_t* out_h;
  float out_h_scale;   // PLAIN: the BF16 output holds y * out_h_scale
  int c_split;         // REC: shuffled channels (16); FUSE: channels of the first part (64)
  int stride2;         // REC: channels per LR pixel of the shuffled tensor (256)
  int r;
  const uint16_t* mask2;  // FUSE n >= c_split: mask at the HR index
  uint16_t* out_h2;       // FUSE n >= c_split: BF16 output at the HR index
};

struct WgradArgs {
  ConvArgs x;            // view of the conv input (mode, tensors, B, H, W, cin_p, taps, kp)
  const uint16_t* dy;    // output gradient, NHWC BF16, dy_stride channels per pixel
  int dy_stride;
  int cout_p;
  int npix;
  int chunk;             // pixels per split (multiple of 32)
  float* part;           // [splits][cout_p][kp]
};

struct NetLayer {
  const char* name;
  int cout, cin, k;
  int cin_p, kp, cout_p;
  int64_t w_off, b_off;  // offsets in the FP32 master vector
  int64_t pk_off;        // offset in the packed BF16 weights
  // data-gradient conv: inputs dY (cinp_t channels stored), outputs cin channels
  int cinp_t, kp_t, coutp_t;
  int64_t pkt_off;       // offset in the packed transposed weights (-1: none)
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
void launch_dgrad(const ConvArgs& a, const BwdEpi& e, int cout_p, hipStream_t st);
void launch_wgrad(const WgradArgs& a, int splits, hipStream_t st);
void launch_bias_partial(const uint16_t* dy, int dy_stride, int cout, int npix, int chunk,
                         int splits, float* bpart, hipStream_t st);
void launch_grad_reduce(const float* part, const float* bpart, int splits, const NetLayer& L,
                        float* g, hipStream_t st);
void launch_pack_t(const float* wm, const NetLayer& L, uint16_t* wt, hipStream_t st);
void launch_l1(const float* y, const float* tgt, int64_t npix, double* part, int nparts,
               double* loss, uint16_t* g8, hipStream_t st);
void launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st);

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
  // training state
  int64_t npacked_t = 0;
  uint16_t* d_packed_t = nullptr;  // transposed weights of the data-gradient convs
  float* d_grad = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  int64_t adam_step = 0;
  char* d_train = nullptr;  // training activations + gradients
  size_t train_bytes = 0;
  double* d_loss = nullptr;
  double* d_lpart = nullptr;
  float* d_wpart = nullptr;
  size_t wpart_floats = 0;
  float* d_bpart = nullptr;
  // views of the last forward's activations (debug)
  int last_B = 0, last_H = 0, last_W = 0;
  float* last_f0 = nullptr;
  float* last_fdf = nullptr;
};
