// Host side of the paper's own fusion network (Sec. 4, Fig. 4): forward,
// training forward and backward.  Kernels are those of cnn.hip; the dense
// connections, the concatenations and the (de)shuffles are all addressing:
//
//  * each residual dense block owns one BF16 tensor D [M][256] holding
//    [x_0 | x_1 | x_2 | x_3]; conv c reads its first 64 (c + 1) channels (a
//    plain view with a pixel stride of 256) and writes x_{c+1} into its slot;
//    the block's last conv writes the block output into slot 0 of the next
//    block's tensor (BF16) and into the FP32 residual stream;
//  * the group and global skips (F_g = chain + F_{g-1}, FDF = F_3 + F0) are
//    extra FP32 residual inputs of that last conv's epilogue;
//  * the stacked stride-2 deshuffle is a view of the fuse conv's input, and
//    each stride-2 shuffle a view of the next conv's input.
//
// Backward: per block, the last conv's data gradient starts an FP32 running
// gradient of slices 0..2 ([M][256]); each earlier conv's data gradient adds
// into the slices it reads, and the one slice no earlier conv reads is then
// complete, goes through its ReLU and becomes the next (earlier) conv's output
// gradient.  The block input's gradient also takes the local skip, and at a
// group's first block the group skip (and at the very first, the global skip
// and F0's ReLU).
#include <cstring>
#include <vector>

#include "mrs_internal.hpp"
#include "cnn.hpp"

namespace mrs {
namespace {

constexpr int NB = RDG_GROUPS * RDG_BLOCKS;

const NetLayer& dense_layer(const mrs_net* net, int g, int b, int c) {
  return net->layers[RDG_L_DENSE + (g * RDG_BLOCKS + b) * RDG_CONVS + c];
}

// Activations of a forward pass.  Inference keeps two dense tensors (the
// current block's and the next one's slot 0); training keeps one per block.
struct RdgActs {
  uint16_t *xh, *xl, *h0, *fl, *fdfh;
  uint16_t* U[RDG_MAX_DSF];  // upscaling step k's ReLU output, 256 channels at LR 2^k
  uint16_t* D[NB];
  float *f0f, *S[2], *F[2], *fdf, *out;
};

// Pixels of the LR image of a net with D stacked deshuffles.
size_t lr_pixels(size_t P, int D) { return P >> (2 * D); }

void plan_acts(std::vector<std::pair<void**, size_t>>& plan, RdgActs& A, size_t P, int D,
               int ndense, bool out) {
  const size_t p = lr_pixels(P, D);
  auto add = [&](void** ptr, size_t bytes) { plan.push_back({ptr, bytes}); };
  add((void**)&A.xh, P * 16 * 2);
  add((void**)&A.xl, p * 8 * 2);
  add((void**)&A.h0, P * NET_FEAT * 2);
  add((void**)&A.fl, p * NET_FEAT * 2);
  add((void**)&A.fdfh, p * NET_FEAT * 2);
  for (int k = 0; k < D; ++k) add((void**)&A.U[k], (p << (2 * k)) * 4 * NET_FEAT * 2);
  for (int i = 0; i < ndense; ++i) add((void**)&A.D[i], p * RDG_DENSE * 2);
  add((void**)&A.f0f, p * NET_FEAT * 4);
  for (int i = 0; i < 2; ++i) add((void**)&A.S[i], p * NET_FEAT * 4);
  for (int i = 0; i < 2; ++i) add((void**)&A.F[i], p * NET_FEAT * 4);
  add((void**)&A.fdf, p * NET_FEAT * 4);
  if (out) add((void**)&A.out, P * 3 * 4);
}

// The whole forward.  `keep`: one dense tensor per block (training); else the
// blocks alternate between D[0] and D[1].
void forward(mrs_net* net, const RdgActs& A, bool keep, int B, int H, int W, const float* hr,
             const float* aux, const float* lr, float* out, hipStream_t st) {
  const std::vector<NetLayer>& Ls = net->layers;
  const int Dn = arch_dsf(net->arch), sc = 1 << Dn;
  const int h = H / sc, w = W / sc;
  const int64_t P = (int64_t)B * H * W, p = (int64_t)lr_pixels(P, Dn);
  prof_begin(KID_CNN_PREP, st);
  launch_prep(net, P, p, hr, aux, lr, A.xh, A.xl, st);
  prof_end(KID_CNN_PREP, st);
  prof_begin(KID_CNN_HR, st);
  {  // F^0_HRLS
    ConvArgs a = base_args(net, Ls[0], B, H, W);
    a.a = A.xh;
    a.ca = 16;
    a.relu = 1;
    a.out_h = A.h0;
    a.out_h_stride = NET_FEAT;
    launch_conv(a, Ls[0].cout_p, st);
  }
  prof_end(KID_CNN_HR, st);
  prof_begin(KID_CNN_LR, st);
  {  // F_LRHS
    ConvArgs a = base_args(net, Ls[1], B, h, w);
    a.a = A.xl;
    a.ca = 8;
    a.relu = 1;
    a.out_h = A.fl;
    a.out_h_stride = NET_FEAT;
    launch_conv(a, Ls[1].cout_p, st);
  }
  {  // F0 = ReLU(fuse [F_LRHS, DSF^D(F^0_HRLS)]) -> FP32 and slot 0 of the first block
    ConvArgs a = base_args(net, Ls[2], B, h, w);
    a.mode = VIEW_CONCAT_UNSHUFFLE;
    a.a = A.fl;
    a.ca = NET_FEAT;
    a.b = A.h0;
    a.cb = NET_FEAT;
    a.r = sc;
    a.dsf = Dn;
    a.relu = 1;
    a.out_f = A.f0f;
    a.out_f_stride = NET_FEAT;
    a.out_h = A.D[0];
    a.out_h_stride = RDG_DENSE;
    launch_conv(a, Ls[2].cout_p, st);
  }
  const float* Fprev = A.f0f;
  int d = 0;
  for (int g = 0; g < RDG_GROUPS; ++g) {
    const float* Sprev = Fprev;
    for (int b = 0; b < RDG_BLOCKS; ++b, ++d) {
      uint16_t* Dc = A.D[keep ? d : (d & 1)];
      for (int c = 0; c < RDG_CONVS - 1; ++c) {  // x_{c+1} = ReLU(conv [x_0 .. x_c])
        const NetLayer& L = dense_layer(net, g, b, c);
        ConvArgs a = base_args(net, L, B, h, w);
        a.a = Dc;
        a.ca = RDG_DENSE;
        a.relu = 1;
        a.out_h = Dc + NET_FEAT * (c + 1);
        a.out_h_stride = RDG_DENSE;
        launch_conv(a, L.cout_p, st);
      }
      // block output = x_0 + conv [x_0 .. x_3] (+ F_{g-1} at a group's end,
      // + F0 at the last group's end, giving FDF)
      const NetLayer& L = dense_layer(net, g, b, RDG_CONVS - 1);
      const bool last = b == RDG_BLOCKS - 1, final_ = last && g == RDG_GROUPS - 1;
      ConvArgs a = base_args(net, L, B, h, w);
      a.a = Dc;
      a.ca = RDG_DENSE;
      a.res = Sprev;
      a.res_scale = 1.0f;
      a.res2 = last ? Fprev : nullptr;
      a.res3 = final_ ? A.f0f : nullptr;
      float* of = final_ ? A.fdf : last ? A.F[g & 1] : A.S[b & 1];
      a.out_f = of;
      a.out_f_stride = NET_FEAT;
      if (final_) {
        a.out_h = A.fdfh;
        a.out_h_stride = NET_FEAT;
      } else {
        a.out_h = A.D[keep ? d + 1 : ((d + 1) & 1)];
        a.out_h_stride = RDG_DENSE;
      }
      launch_conv(a, L.cout_p, st);
      Sprev = of;
      if (last) Fprev = of;
    }
  }
  for (int k = 0; k < Dn; ++k) {  // U_k = ReLU(conv (k ? shuffle2(U_{k-1}) : FDF)), 256 ch
    const NetLayer& Lu = Ls[RDG_L_UP + k];
    ConvArgs a = base_args(net, Lu, B, h << k, w << k);
    if (k == 0) {
      a.a = A.fdfh;
      a.ca = NET_FEAT;
    } else {
      a.mode = VIEW_SHUFFLE_CONCAT;
      a.a = A.U[k - 1];
      a.ca = 4 * NET_FEAT;
      a.c0 = NET_FEAT;
      a.r = 2;
    }
    a.relu = 1;
    a.out_h = A.U[k];
    a.out_h_stride = Lu.cout;
    launch_conv(a, Lu.cout_p, st);
  }
  prof_end(KID_CNN_LR, st);
  prof_begin(KID_CNN_REC, st);
  {  // I_SR = conv shuffle2(U_{D-1})
    const NetLayer& Lr = Ls[RDG_L_UP + Dn];
    ConvArgs a = base_args(net, Lr, B, H, W);
    a.mode = VIEW_SHUFFLE_CONCAT;
    a.a = A.U[Dn - 1];
    a.ca = 4 * NET_FEAT;
    a.c0 = NET_FEAT;
    a.r = 2;
    a.out_f = out;
    a.out_f_stride = 3;
    launch_conv(a, Lr.cout_p, st);
  }
  prof_end(KID_CNN_REC, st);
}

// Gradient buffers of the backward pass.
struct RdgGrads {
  uint16_t *g8, *dfdfh, *dFh[2], *dsh[2], *dy[2], *df0h, *dflh, *dh0h;
  uint16_t* dU[RDG_MAX_DSF];
  float *dfdf, *dF[2], *dsf[2], *ga;
};

void plan_grads(std::vector<std::pair<void**, size_t>>& plan, RdgGrads& G, size_t P, int D) {
  const size_t p = lr_pixels(P, D);
  auto add = [&](void** ptr, size_t bytes) { plan.push_back({ptr, bytes}); };
  add((void**)&G.g8, P * 8 * 2);
  for (int k = 0; k < D; ++k) add((void**)&G.dU[k], (p << (2 * k)) * 4 * NET_FEAT * 2);
  add((void**)&G.dfdfh, p * NET_FEAT * 2);
  for (int i = 0; i < 2; ++i) {
    add((void**)&G.dFh[i], p * NET_FEAT * 2);
    add((void**)&G.dsh[i], p * NET_FEAT * 2);
    add((void**)&G.dy[i], p * NET_FEAT * 2);
    add((void**)&G.dF[i], p * NET_FEAT * 4);
    add((void**)&G.dsf[i], p * NET_FEAT * 4);
  }
  add((void**)&G.df0h, p * NET_FEAT * 2);
  add((void**)&G.dflh, p * NET_FEAT * 2);
  add((void**)&G.dh0h, P * NET_FEAT * 2);
  add((void**)&G.dfdf, p * NET_FEAT * 4);
  add((void**)&G.ga, p * RDG_DENSE * 4);
}

ConvArgs dense_view(const mrs_net* net, const NetLayer& L, int B, int h, int w,
                    const uint16_t* D) {
  ConvArgs x = base_args(net, L, B, h, w);
  x.a = D;
  x.ca = RDG_DENSE;
  return x;
}

// The input view of upscaling step k (k >= 1) or of the reconstruction conv
// (k = D): shuffle2 of U_{k-1}, at LR resolution x 2^k.
ConvArgs shuffle_view(const mrs_net* net, const NetLayer& L, int B, int hk, int wk,
                      const uint16_t* U) {
  ConvArgs x = base_args(net, L, B, hk, wk);
  x.mode = VIEW_SHUFFLE_CONCAT;
  x.a = U;
  x.ca = 4 * NET_FEAT;
  x.c0 = NET_FEAT;
  x.r = 2;
  return x;
}

void backward(mrs_net* net, const RdgActs& A, const RdgGrads& G, int B, int H, int W,
              hipStream_t st) {
  const std::vector<NetLayer>& Ls = net->layers;
  const int Dn = arch_dsf(net->arch), sc = 1 << Dn;
  const int h = H / sc, w = W / sc;
  // rec (k = D) and upscaling steps D-1 .. 1: d shuffle2(U_{k-1}) -> dU_{k-1}
  // (masked by U_{k-1} > 0, stored like U_{k-1})
  for (int k = Dn; k >= 1; --k) {
    const NetLayer& L = Ls[RDG_L_UP + k];
    const int hk = h << k, wk = w << k;
    const uint16_t* dy = k == Dn ? G.g8 : G.dU[k];
    const int dy_stride = k == Dn ? 8 : L.cout;
    ConvArgs a = tconv_args(net, L, B, hk, wk, dy);
    BwdEpi e = plain_epi();
    e.mode = EPI_REC_SPLIT;
    e.out_h = G.dU[k - 1];
    e.mask = A.U[k - 1];
    e.c_split = NET_FEAT;
    e.stride2 = 4 * NET_FEAT;
    e.r = 2;
    launch_dgrad(a, e, L.coutp_t, st);
    wgrad(net, L, shuffle_view(net, L, B, hk, wk, A.U[k - 1]), dy, dy_stride, st);
  }
  {  // up0: dFDF (FP32 + BF16)
    const NetLayer& Lu0 = Ls[RDG_L_UP];
    ConvArgs a = tconv_args(net, Lu0, B, h, w, G.dU[0]);
    BwdEpi e = plain_epi();
    e.out_f = G.dfdf;
    e.out_h = G.dfdfh;
    launch_dgrad(a, e, Lu0.coutp_t, st);
    ConvArgs x = base_args(net, Lu0, B, h, w);
    x.a = A.fdfh;
    x.ca = NET_FEAT;
    wgrad(net, Lu0, x, G.dU[0], Lu0.cout, st);
  }
  // groups, last to first; dF = gradient of F_g (the group's output)
  const float* dFf = G.dfdf;
  const uint16_t* dFh = G.dfdfh;
  for (int g = RDG_GROUPS - 1; g >= 0; --g) {
    const float* dsf = dFf;  // gradient of the chain's end = of F_g
    const uint16_t* dsh = dFh;
    for (int b = RDG_BLOCKS - 1; b >= 0; --b) {
      const uint16_t* D = A.D[g * RDG_BLOCKS + b];
      for (int c = RDG_CONVS - 1; c >= 0; --c) {
        const NetLayer& L = dense_layer(net, g, b, c);
        const bool fusing = c == RDG_CONVS - 1;
        // output gradient of conv c: the block output's for the fusing conv,
        // else the one the later conv completed (dy ping-pong)
        const uint16_t* dy = fusing ? dsh : G.dy[(c + 1) & 1];
        ConvArgs a = tconv_args(net, L, B, h, w, dy);
        BwdEpi e = plain_epi();
        e.mode = EPI_DENSE;
        e.k = c + 1;
        e.fusing = fusing;
        e.ga = G.ga;
        e.ds = dsf;
        e.dense = D;
        if (c > 0) {
          e.dy_next = G.dy[c & 1];
        } else {  // block input: + local skip (in ga), + group skip, + global skip
          const bool first = b == 0;
          e.add1 = first ? dFf : nullptr;
          e.add2 = (first && g == 0) ? G.dfdf : nullptr;
          e.mask0 = first && g == 0;
          if (first && g == 0) {
            e.out_f = nullptr;
            e.out_h = G.df0h;
          } else if (first) {
            e.out_f = G.dF[g & 1];
            e.out_h = G.dFh[g & 1];
          } else {
            e.out_f = G.dsf[b & 1];
            e.out_h = G.dsh[b & 1];
          }
        }
        launch_dgrad(a, e, L.coutp_t, st);
        wgrad(net, L, dense_view(net, L, B, h, w, D), dy, NET_FEAT, st);
      }
      if (b > 0) {
        dsf = G.dsf[b & 1];
        dsh = G.dsh[b & 1];
      }
    }
    if (g > 0) {
      dFf = G.dF[g & 1];
      dFh = G.dFh[g & 1];
    }
  }
  {  // fuse: d[fl, DSF^D(h0)] -> dfl (masked) and dh0 (masked), no other use of h0
    const NetLayer& Lf = Ls[2];
    ConvArgs a = tconv_args(net, Lf, B, h, w, G.df0h);
    BwdEpi e = plain_epi();
    e.mode = EPI_FUSE_SPLIT;
    e.c_split = NET_FEAT;
    e.stride = NET_FEAT;
    e.mask = A.fl;
    e.out_h = G.dflh;
    e.mask2 = A.h0;
    e.out_h2 = G.dh0h;
    e.r = sc;
    e.dsf = Dn;
    launch_dgrad(a, e, Lf.coutp_t, st);
    ConvArgs x = base_args(net, Lf, B, h, w);
    x.mode = VIEW_CONCAT_UNSHUFFLE;
    x.a = A.fl;
    x.ca = NET_FEAT;
    x.b = A.h0;
    x.cb = NET_FEAT;
    x.r = sc;
    x.dsf = Dn;
    wgrad(net, Lf, x, G.df0h, NET_FEAT, st);
  }
  {  // encoders: weight gradients only
    ConvArgs x = base_args(net, Ls[1], B, h, w);
    x.a = A.xl;
    x.ca = 8;
    wgrad(net, Ls[1], x, G.dflh, NET_FEAT, st);
    x = base_args(net, Ls[0], B, H, W);
    x.a = A.xh;
    x.ca = 16;
    wgrad(net, Ls[0], x, G.dh0h, NET_FEAT, st);
  }
}

}  // namespace

mrs_status rdg_forward(mrs_net* net, int B, int H, int W, const float* hr, const float* aux,
                       const float* lr, float* out, hipStream_t st) {
  RdgActs A;
  std::memset(&A, 0, sizeof A);
  std::vector<std::pair<void**, size_t>> plan;
  plan_acts(plan, A, (size_t)B * H * W, arch_dsf(net->arch), 2, false);
  mrs_status rc = arena_carve(net->d_arena, net->arena_bytes, plan, st, "mrs_fuse");
  if (rc != MRS_OK) return rc;
  forward(net, A, false, B, H, W, hr, aux, lr, out, st);
  MRS_TRY_HIP(hipGetLastError());
  net->last_B = B;
  net->last_H = H;
  net->last_W = W;
  net->last_f0 = A.f0f;
  net->last_fdf = A.fdf;
  return MRS_OK;
}

mrs_status rdg_loss_grad(mrs_net* net, int B, int H, int W, const float* hr, const float* aux,
                         const float* lr, const OutGrad& og, const float** out, hipStream_t st) {
  RdgActs A;
  RdgGrads G;
  std::memset(&A, 0, sizeof A);
  std::memset(&G, 0, sizeof G);
  const size_t P = (size_t)B * H * W;
  std::vector<std::pair<void**, size_t>> plan;
  plan_acts(plan, A, P, arch_dsf(net->arch), NB, true);
  plan_grads(plan, G, P, arch_dsf(net->arch));
  mrs_status rc = arena_carve(net->d_train, net->train_bytes, plan, st, "mrs_train_step");
  if (rc != MRS_OK) return rc;
  rc = ensure_wpart(net, (int64_t)P, st);
  if (rc != MRS_OK) return rc;
  prof_begin(KID_TRAIN_FWD, st);
  forward(net, A, true, B, H, W, hr, aux, lr, A.out, st);
  prof_end(KID_TRAIN_FWD, st);
  launch_out_grad(og, A.out, (int64_t)P, G.g8, st);
  prof_begin(KID_TRAIN_BWD, st);
  backward(net, A, G, B, H, W, st);
  prof_end(KID_TRAIN_BWD, st);
  MRS_TRY_HIP(hipGetLastError());
  *out = A.out;
  return MRS_OK;
}

}  // namespace mrs
