// Fusion-network internals shared by cnn.hip (kernels) and net.hip (host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
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
  int dsf;  // CONCAT_UNSHUFFLE: 0 = one stride-r unshuffle, D = D stacked stride-2 (r = 2^D)
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
  const float* res3;  // optional FP32 [M][cout]: y += res3
  float* out_f;       // optional FP32 output, out_f_stride floats per pixel
  int out_f_stride;
  uint16_t* out_h;  // optional BF16 output, out_h_stride per pixel
  int out_h_stride;
};

enum EpiMode { EPI_PLAIN = 0, EPI_REC_SPLIT = 1, EPI_FUSE_SPLIT = 2, EPI_DENSE = 3 };

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
  int dsf;                // FUSE: as ConvArgs::dsf
  // DENSE: data gradient of the conv of a residual dense block that reads the
  // first k 64-channel slices of the block's dense tensor [x_0 .. x_3].
  int k;
  int fusing;             // the block's last conv: starts the slice gradients
  float* ga;              // FP32 [M][256] running gradients of slices 0 .. k-2
  const float* ds;        // fusing: dL/d(block output) [M][64], the local skip's share of x_0
  const uint16_t* dense;  // the block's dense tensor BF16 [M][256] (ReLU masks)
  uint16_t* dy_next;      // k >= 2: BF16 [M][64] gradient of x_{k-1} at its conv's output
  int mask0;              // k == 1: x_0 is a ReLU output (F_0): mask by it
  // k == 1: dL/dx_0 = ga + acc + add1 + add2 -> out_f (FP32 [M][64], optional), out_h (BF16)
};

struct WgradArgs {
  ConvArgs x;            // view of the conv input (mode, tensors, B, H, W, cin_p, taps, kp)
  const uint16_t* dy;    // output gradient, NHWC BF16, dy_stride channels per pixel
  int dy_stride;
  int cout_p;
  int npix;
  int chunk;             // pixels per split (multiple of 128)
  float* part;           // [splits][cout_p][kp]
  int cout;              // output channels with a bias
  float* bpart;          // [splits][cout]: the bias gradient's partial sums
};

// How a backward pass gets its output gradient dL/dI_SR: from a loss of the
// output against `tgt` (beta 0: L1, > 0: the robust loss; FP64 value in
// *loss), or (tgt NULL) as given by the caller in `gout` (FP32 [P][3]).
struct OutGrad {
  const float* tgt;
  float beta;
  const float* gout;
  double* part;
  int nparts;
  double* loss;
};
struct NetLayer {
  const char* name;
  int cout, cin, k;
  int level;         // resolution: 0 HR, 1 HR/2, 2 LR (HR/4)
  float init_scale;  // multiplies the He-uniform bound
  int cin_p, kp, cout_p;
  int64_t w_off, b_off;  // offsets in the FP32 master vector
  int64_t pk_off;        // offset in the packed BF16 weights
  // data-gradient conv: inputs dY (cinp_t channels stored), outputs cin channels
  int cinp_t, kp_t, coutp_t;
  int64_t pkt_off;       // offset in the packed transposed weights (-1: none)
};

// One layer's BF16 packing job of k_pack_all: the forward layout (t = 0) or
// the transposed layout of its data-gradient conv (t = 1).
struct PackJob {
  int64_t begin;    // index of the job's first element in the launch
  int64_t w_off;    // the layer's FP32 master weights
  int64_t out_off;  // offset in d_packed (t = 0) or d_packed_t (t = 1)
  int cout, cin, ksz;
  int cinp, kp, coutp;  // padded layout of the output
  int t;
};

constexpr int NET_FEAT = 64;
constexpr int NET_SCALE = 4;
constexpr int NET_NRES = 16;
constexpr int NET_UPCH = 16;
constexpr float NET_RES_SCALE = 0.1f;
constexpr int64_t NET_NUM_PARAMS = 1408883;

// The paper's own network (Sec. 4): G residual dense groups of B blocks of 4
// densely connected convs (growth 64), two stacked stride-2 deshuffles, two
// stride-2 sub-pixel upscaling steps.
constexpr int RDG_GROUPS = 3;
constexpr int RDG_BLOCKS = 5;
constexpr int RDG_CONVS = 4;
constexpr int RDG_DENSE = NET_FEAT * RDG_CONVS;  // channels of a block's dense tensor
constexpr int RDG_L_DENSE = 3;                                             // first dense conv
constexpr int RDG_L_UP = RDG_L_DENSE + RDG_GROUPS * RDG_BLOCKS * RDG_CONVS;  // up0.., rec
constexpr int RDG_MAX_DSF = 3;
// scale (2, 4 or 8) of an architecture; D = log2(scale) for the dense-group nets
int arch_scale(int arch);
int arch_dsf(int arch);
bool arch_is_rdg(int arch);
bool arch_has_layers(int arch);  // HRLS input with the render layers (16 channels)

std::vector<NetLayer> make_layers(int arch);
size_t align256(size_t v);
ConvArgs base_args(const mrs_net* net, const NetLayer& L, int B, int H, int W);
ConvArgs tconv_args(const mrs_net* net, const NetLayer& L, int B, int H, int W,
                    const uint16_t* dy);
BwdEpi plain_epi();
void wgrad(mrs_net* net, const NetLayer& L, const ConvArgs& x, const uint16_t* dy, int dy_stride,
           hipStream_t st);
int wgrad_splits(int64_t npix, int kp, int cout_p, int& chunk);
// Split-K partial buffers for the weight gradients at P HR pixels.
mrs_status ensure_wpart(mrs_net* net, int64_t P, hipStream_t st);
// The paper's network (net_rdg.hip): forward into out; forward + output
// gradient + backward into net->d_grad, *out = the network output.
mrs_status rdg_forward(mrs_net* net, int B, int H, int W, const float* hr, const float* aux,
                       const float* lr, float* out, hipStream_t st);
mrs_status rdg_loss_grad(mrs_net* net, int B, int H, int W, const float* hr, const float* aux,
                         const float* lr, const OutGrad& og, const float** out, hipStream_t st);
// Carves `plan` (pointer, bytes) out of one device allocation, growing it if needed.
mrs_status arena_carve(char*& base, size_t& cap, std::vector<std::pair<void**, size_t>>& plan,
                       hipStream_t st, const char* what);

void launch_conv(const ConvArgs& a, int cout_p, hipStream_t st);
// a then b as one residual block (k_res_block) when both are 3x3 64 -> 64
// convs over the same plain BF16 input grid and a has the ReLU; false (nothing
// launched) otherwise.
bool launch_res_block(const ConvArgs& a, const ConvArgs& b, hipStream_t st);
void launch_prep(const mrs_net* net, int64_t nhr, int64_t nlr, const float* hr, const float* aux,
                 const float* lr, uint16_t* xh, uint16_t* xl, hipStream_t st);
void launch_init(float* dst, const NetLayer& L, uint64_t seed, hipStream_t st);
void launch_dgrad(const ConvArgs& a, const BwdEpi& e, int cout_p, hipStream_t st);
void launch_wgrad(const WgradArgs& a, int splits, hipStream_t st);
void launch_grad_reduce(const float* part, const float* bpart, int splits, const NetLayer& L,
                        float* g, hipStream_t st);
void launch_pack_all(const float* wm, const PackJob* jobs, int njobs, int64_t total,
                     uint16_t* packed, uint16_t* packed_t, hipStream_t st);
void launch_out_grad(const OutGrad& o, const float* y, int64_t npix, uint16_t* g8,
                     hipStream_t st);
void launch_sgd(float* w, const float* g, int64_t n, float lr, hipStream_t st);
void launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st);

}  // namespace mrs

struct mrs_net {
  int arch = 0;  // MRS_NET_*
  // render layers of the HRLS input, bound by mrs_net_bind_layers (layered archs)
  const float* in_layers = nullptr;
  const float* in_sumsq = nullptr;
  int32_t in_spp = 0;
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
  // packing jobs of every layer (forward layouts, then transposed), on device
  mrs::PackJob* d_packjobs = nullptr;
  int packjobs_fwd = 0, packjobs_all = 0;
  int64_t pack_total_fwd = 0, pack_total_all = 0;
  // views of the last forward's activations (debug)
  int last_B = 0, last_H = 0, last_W = 0;
  float* last_f0 = nullptr;
  float* last_fdf = nullptr;
};
