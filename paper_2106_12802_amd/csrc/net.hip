// Host side of the fusion network: layer table, parameters, forward pass.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mrs_internal.hpp"
#include "cnn.hpp"

namespace mrs {
namespace {

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Spec {
  const char* name;
  int cout, cin, k, cin_p, level;
  float init_scale;
};

// Layer list of the 16-residual-block network; hr_in HRLS input channels (10,
// or 16 with the render layers), padded to 16.
std::vector<Spec> specs_res16(int hr_in) {
  static std::vector<std::string> names;
  std::vector<Spec> specs = {{"hrls", NET_FEAT, hr_in, 3, 16, 0, 1.0f},
                             {"lrhs", NET_FEAT, 3, 3, 8, 2, 1.0f},
                             {"fuse", NET_FEAT, NET_FEAT + NET_SCALE * NET_SCALE * NET_FEAT, 1,
                              NET_FEAT + NET_SCALE * NET_SCALE * NET_FEAT, 2, 1.0f}};
  if (names.empty()) {
    for (int i = 0; i < NET_NRES; ++i) {
      names.push_back("res" + std::to_string(i) + "a");
      names.push_back("res" + std::to_string(i) + "b");
    }
  }
  for (int i = 0; i < 2 * NET_NRES; ++i)
    specs.push_back({names[i].c_str(), NET_FEAT, NET_FEAT, 3, NET_FEAT, 2, 1.0f});
  specs.push_back({"up", NET_UPCH * NET_SCALE * NET_SCALE, NET_FEAT, 3, NET_FEAT, 2, 1.0f});
  specs.push_back({"rec", 3, NET_UPCH + NET_FEAT, 3, NET_UPCH + NET_FEAT, 0, 1.0f});
  return specs;
}

// Layer list of the paper's network (Sec. 4): encoders, 1x1 fuse, G x B residual
// dense blocks of 4 convs (conv c reads 64 (c + 1) channels; the fourth fuses
// them back to 64 and feeds the block's skip, its initial weights scaled by 0.1
// so that the chain of 15 skips starts near the identity), two stride-2
// upscaling convs, reconstruction (also scaled by 0.1, so that the first
// outputs are near the scale of the images rather than ~10x above it, where
// the robust loss is flat and training drifts away).
// D = log2(scale) stacked stride-2 deshuffles and as many upscaling steps.
std::vector<Spec> specs_rdg(int D, int hr_in) {
  static std::vector<std::string> names;
  if (names.empty()) {
    for (int g = 0; g < RDG_GROUPS; ++g)
      for (int b = 0; b < RDG_BLOCKS; ++b)
        for (int c = 0; c < RDG_CONVS; ++c)
          names.push_back("g" + std::to_string(g) + "b" + std::to_string(b) + "c" +
                          std::to_string(c));
    for (int k = 0; k < RDG_MAX_DSF; ++k) names.push_back("up" + std::to_string(k));
  }
  const int fuse_in = NET_FEAT + (1 << (2 * D)) * NET_FEAT;
  std::vector<Spec> specs = {{"hrls", NET_FEAT, hr_in, 3, 16, 0, 1.0f},
                             {"lrhs", NET_FEAT, 3, 3, 8, D, 1.0f},
                             {"fuse", NET_FEAT, fuse_in, 1, fuse_in, D, 1.0f}};
  const int ndense = RDG_GROUPS * RDG_BLOCKS * RDG_CONVS;
  for (int i = 0; i < ndense; ++i) {
    const int c = i % RDG_CONVS, cin = NET_FEAT * (c + 1);
    specs.push_back({names[i].c_str(), NET_FEAT, cin, 3, cin, D,
                     c == RDG_CONVS - 1 ? 0.1f : 1.0f});
  }
  for (int k = 0; k < D; ++k)  // step k runs at HR / 2^(D - k)
    specs.push_back({names[ndense + k].c_str(), 4 * NET_FEAT, NET_FEAT, 3, NET_FEAT, D - k, 1.0f});
  specs.push_back({"rec", 3, NET_FEAT, 3, NET_FEAT, 0, 0.1f});
  return specs;
}

}  // namespace

int arch_scale(int arch) {
  return arch == MRS_NET_RDG_X2 ? 2 : arch == MRS_NET_RDG_X8 ? 8 : 4;
}

int arch_dsf(int arch) {
  return arch == MRS_NET_RDG_X2 ? 1 : arch == MRS_NET_RDG_X8 ? 3 : 2;
}

bool arch_is_rdg(int arch) {
  return arch == MRS_NET_RDG || arch == MRS_NET_RDG_X2 || arch == MRS_NET_RDG_X8 ||
         arch == MRS_NET_RDG_LAYERS;
}

bool arch_has_layers(int arch) {
  return arch == MRS_NET_RES16_LAYERS || arch == MRS_NET_RDG_LAYERS;
}

bool arch_known(int arch) { return arch == MRS_NET_RES16 || arch == MRS_NET_RES16_LAYERS || arch_is_rdg(arch); }

std::vector<NetLayer> make_layers(int arch) {
  const int hr_in = arch_has_layers(arch) ? 16 : 10;
  const std::vector<Spec> specs =
      arch_is_rdg(arch) ? specs_rdg(arch_dsf(arch), hr_in) : specs_res16(hr_in);
  std::vector<NetLayer> L;
  int64_t off = 0, pk = 0, pkt = 0;
  for (const Spec& s : specs) {
    NetLayer l;
    l.name = s.name;
    l.cout = s.cout;
    l.cin = s.cin;
    l.k = s.k;
    l.level = s.level;
    l.init_scale = s.init_scale;
    l.cin_p = s.cin_p;
    l.kp = round_up(s.k * s.k * s.cin_p, 32);
    l.cout_p = s.cout >= 64 ? round_up(s.cout, 64) : round_up(s.cout, 16);
    l.w_off = off;
    off += (int64_t)s.cout * s.cin * s.k * s.k;
    l.b_off = off;
    off += s.cout;
    l.pk_off = pk;
    pk += (int64_t)l.cout_p * l.kp;
    // data-gradient conv: reads dY with the channel count it is stored with
    const std::string nm = s.name;
    if (nm == "hrls" || nm == "lrhs") {
      l.cinp_t = l.kp_t = l.coutp_t = 0;
      l.pkt_off = -1;
    } else {
      l.cinp_t = nm == "rec" ? 8 : s.cout;
      l.kp_t = round_up(s.k * s.k * l.cinp_t, 32);
      l.coutp_t = s.cin >= 64 ? round_up(s.cin, 64) : round_up(s.cin, 16);
      l.pkt_off = pkt;
      pkt += (int64_t)l.coutp_t * l.kp_t;
    }
    L.push_back(l);
  }
  return L;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

mrs_status arena_carve(char*& base, size_t& cap, std::vector<std::pair<void**, size_t>>& plan,
                       hipStream_t st, const char* what) {
  size_t total = 0;
  for (auto& e : plan) total += align256(e.second);
  if (total > cap) {
    if (base) {
      MRS_TRY_HIP(hipStreamSynchronize(st));
      (void)hipFree(base);
    }
    base = nullptr;
    cap = 0;
    if (hipMalloc(&base, total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MRS_ERR_OUT_OF_MEMORY, std::string(what) + ": device allocation failed");
    }
    cap = total;
  }
  size_t off = 0;
  for (auto& e : plan) {
    *e.first = base + off;
    off += align256(e.second);
  }
  return MRS_OK;
}

namespace {

struct Arena {
  uint16_t *xh, *xl, *h0, *fl, *f0h, *rh[2], *th, *U;
  float *f0f, *rf[2];
};

mrs_status ensure_arena(mrs_net* net, int B, int H, int W, Arena& A) {
  const size_t P = (size_t)B * H * W, p = P / 16;
  std::vector<std::pair<void**, size_t>> plan = {
      {(void**)&A.xh, P * 16 * 2},   {(void**)&A.xl, p * 8 * 2},    {(void**)&A.h0, P * 64 * 2},
      {(void**)&A.fl, p * 64 * 2},   {(void**)&A.f0f, p * 64 * 4},  {(void**)&A.f0h, p * 64 * 2},
      {(void**)&A.rf[0], p * 64 * 4}, {(void**)&A.rf[1], p * 64 * 4},
      {(void**)&A.rh[0], p * 64 * 2}, {(void**)&A.rh[1], p * 64 * 2},
      {(void**)&A.th, p * 64 * 2},   {(void**)&A.U, p * 256 * 2}};
  return arena_carve(net->d_arena, net->arena_bytes, plan, current_stream(), "mrs_fuse");
}

}  // namespace

ConvArgs base_args(const mrs_net* net, const NetLayer& L, int B, int H, int W) {
  ConvArgs a;
  std::memset(&a, 0, sizeof a);
  a.mode = VIEW_PLAIN;
  a.B = B;
  a.H = H;
  a.W = W;
  a.cin_p = L.cin_p;
  a.taps = L.k * L.k;
  a.kp = L.kp;
  a.w = net->d_packed + L.pk_off;
  a.bias = net->d_master + L.b_off;
  a.cout = L.cout;
  a.res_scale = 1.0f;
  return a;
}

mrs_status net_forward(mrs_net* net, int B, int H, int W, const float* hr, const float* aux,
                       const float* lr, float* out, hipStream_t st) {
  Arena A;
  mrs_status rc = ensure_arena(net, B, H, W, A);
  if (rc != MRS_OK) return rc;
  const std::vector<NetLayer>& Ls = net->layers;
  const int h = H / NET_SCALE, w = W / NET_SCALE;
  const int64_t P = (int64_t)B * H * W, p = P / 16;
  prof_begin(KID_CNN_PREP, st);
  launch_prep(net, P, p, hr, aux, lr, A.xh, A.xl, st);
  prof_end(KID_CNN_PREP, st);
  prof_begin(KID_CNN_HR, st);
  {  // h0 = ReLU(conv(xh))
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
  {  // fl = ReLU(conv(xl))
    ConvArgs a = base_args(net, Ls[1], B, h, w);
    a.a = A.xl;
    a.ca = 8;
    a.relu = 1;
    a.out_h = A.fl;
    a.out_h_stride = NET_FEAT;
    launch_conv(a, Ls[1].cout_p, st);
  }
  {  // F0 = ReLU(conv1x1([fl, unshuffle(h0)]))
    ConvArgs a = base_args(net, Ls[2], B, h, w);
    a.mode = VIEW_CONCAT_UNSHUFFLE;
    a.a = A.fl;
    a.ca = NET_FEAT;
    a.b = A.h0;
    a.cb = NET_FEAT;
    a.r = NET_SCALE;
    a.relu = 1;
    a.out_f = A.f0f;
    a.out_f_stride = NET_FEAT;
    a.out_h = A.f0h;
    a.out_h_stride = NET_FEAT;
    launch_conv(a, Ls[2].cout_p, st);
  }
  const float* cur_f = A.f0f;
  const uint16_t* cur_h = A.f0h;
  for (int i = 0; i < NET_NRES; ++i) {
    const NetLayer& La = Ls[3 + 2 * i];
    const NetLayer& Lb = Ls[4 + 2 * i];
    ConvArgs a = base_args(net, La, B, h, w);
    a.a = cur_h;
    a.ca = NET_FEAT;
    a.relu = 1;
    a.out_h = A.th;
    a.out_h_stride = NET_FEAT;
    ConvArgs bb = base_args(net, Lb, B, h, w);
    bb.a = A.th;
    bb.ca = NET_FEAT;
    bb.res = cur_f;
    bb.res_scale = NET_RES_SCALE;
    bb.res2 = (i == NET_NRES - 1) ? A.f0f : nullptr;  // F_DF = r_16 + F_0
    bb.out_f = A.rf[i & 1];
    bb.out_f_stride = NET_FEAT;
    bb.out_h = A.rh[i & 1];
    bb.out_h_stride = NET_FEAT;
    // both convs in one launch (bitwise the same), or one after the other
    // through the BF16 intermediate A.th; small images (fewer 16x16 tiles than
    // the small-tile threshold) keep the two convs, whose small-tile plan
    // spreads them over more blocks
    const int64_t tiles = (int64_t)B * ((h + 15) / 16) * ((w + 15) / 16);
    if (!(net_fused_blocks() && tiles >= conv_small_tiles() && launch_res_block(a, bb, st))) {
      launch_conv(a, La.cout_p, st);
      launch_conv(bb, Lb.cout_p, st);
    }
    cur_f = A.rf[i & 1];
    cur_h = A.rh[i & 1];
  }
  const NetLayer& Lu = Ls[3 + 2 * NET_NRES];
  const NetLayer& Lr = Ls[4 + 2 * NET_NRES];
  {  // U = ReLU(conv(FDF)), 256 channels at LR
    ConvArgs a = base_args(net, Lu, B, h, w);
    a.a = cur_h;
    a.ca = NET_FEAT;
    a.relu = 1;
    a.out_h = A.U;
    a.out_h_stride = Lu.cout;
    launch_conv(a, Lu.cout_p, st);
  }
  prof_end(KID_CNN_LR, st);
  prof_begin(KID_CNN_REC, st);
  {  // out = conv([shuffle(U), h0])
    ConvArgs a = base_args(net, Lr, B, H, W);
    a.mode = VIEW_SHUFFLE_CONCAT;
    a.a = A.U;
    a.ca = Lu.cout;
    a.c0 = NET_UPCH;
    a.r = NET_SCALE;
    a.b = A.h0;
    a.cb = NET_FEAT;
    a.out_f = out;
    a.out_f_stride = 3;
    launch_conv(a, Lr.cout_p, st);
  }
  prof_end(KID_CNN_REC, st);
  MRS_TRY_HIP(hipGetLastError());
  net->last_B = B;
  net->last_H = H;
  net->last_W = W;
  net->last_f0 = A.f0f;
  net->last_fdf = const_cast<float*>(cur_f);
  return MRS_OK;
}

// The table of packing jobs (built once: forward layouts of every layer, then
// the transposed layouts of those with a data-gradient conv).
mrs_status ensure_pack_jobs(mrs_net* net) {
  if (net->d_packjobs) return MRS_OK;
  std::vector<PackJob> jobs;
  int64_t at = 0;
  for (int t = 0; t < 2; ++t) {
    for (const NetLayer& L : net->layers) {
      if (t == 1 && L.pkt_off < 0) continue;
      PackJob j;
      j.begin = at;
      j.w_off = L.w_off;
      j.out_off = t ? L.pkt_off : L.pk_off;
      j.cout = L.cout;
      j.cin = L.cin;
      j.ksz = L.k;
      j.cinp = t ? L.cinp_t : L.cin_p;
      j.kp = t ? L.kp_t : L.kp;
      j.coutp = t ? L.coutp_t : L.cout_p;
      j.t = t;
      jobs.push_back(j);
      at += (int64_t)j.coutp * j.kp;
    }
    if (t == 0) {
      net->packjobs_fwd = (int)jobs.size();
      net->pack_total_fwd = at;
    }
  }
  net->packjobs_all = (int)jobs.size();
  net->pack_total_all = at;
  if (hipMalloc(&net->d_packjobs, sizeof(PackJob) * jobs.size()) != hipSuccess) {
    (void)hipGetLastError();
    net->d_packjobs = nullptr;
    return fail(MRS_ERR_OUT_OF_MEMORY, "packing table allocation failed");
  }
  MRS_TRY_HIP(hipMemcpy(net->d_packjobs, jobs.data(), sizeof(PackJob) * jobs.size(),
                        hipMemcpyHostToDevice));
  return MRS_OK;
}

mrs_status net_refresh_packed(mrs_net* net, hipStream_t st) {
  mrs_status rc = ensure_pack_jobs(net);
  if (rc != MRS_OK) return rc;
  const bool with_t = net->d_packed_t != nullptr;
  launch_pack_all(net->d_master, net->d_packjobs, with_t ? net->packjobs_all : net->packjobs_fwd,
                  with_t ? net->pack_total_all : net->pack_total_fwd, net->d_packed,
                  net->d_packed_t, st);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

// ------------------------------------------------------------------ training

// Split-K partial buffers for the weight gradients of every layer at batch
// size B x H x W (pixel count per layer from its resolution level).
mrs_status ensure_wpart(mrs_net* net, int64_t P, hipStream_t st) {
  size_t need_w = 0, need_b = 0;
  for (const NetLayer& L : net->layers) {
    int chunk;
    const int sp = wgrad_splits(P >> (2 * L.level), L.kp, L.cout_p, chunk);
    need_w = std::max(need_w, (size_t)sp * L.cout_p * L.kp);
    need_b = std::max(need_b, (size_t)sp * L.cout);
  }
  if (need_w > net->wpart_floats) {
    if (net->d_wpart) {
      MRS_TRY_HIP(hipStreamSynchronize(st));
      (void)hipFree(net->d_wpart);
      (void)hipFree(net->d_bpart);
    }
    net->d_wpart = nullptr;
    net->d_bpart = nullptr;
    net->wpart_floats = 0;
    if (hipMalloc(&net->d_wpart, sizeof(float) * need_w) != hipSuccess ||
        hipMalloc(&net->d_bpart, sizeof(float) * std::max<size_t>(need_b, 256 * 256)) !=
            hipSuccess) {
      (void)hipGetLastError();
      return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_train_step: gradient scratch allocation failed");
    }
    net->wpart_floats = need_w;
  }
  return MRS_OK;
}

void wgrad(mrs_net* net, const NetLayer& L, const ConvArgs& x, const uint16_t* dy, int dy_stride,
           hipStream_t st) {
  WgradArgs w;
  w.x = x;
  w.dy = dy;
  w.dy_stride = dy_stride;
  w.cout_p = L.cout_p;
  w.npix = x.B * x.H * x.W;
  const int splits = wgrad_splits(w.npix, L.kp, L.cout_p, w.chunk);
  w.part = net->d_wpart;
  w.cout = L.cout;
  w.bpart = net->d_bpart;
  launch_wgrad(w, splits, st);
  launch_grad_reduce(net->d_wpart, net->d_bpart, splits, L, net->d_grad + L.w_off, st);
}

ConvArgs tconv_args(const mrs_net* net, const NetLayer& L, int B, int H, int W,
                    const uint16_t* dy) {
  ConvArgs a;
  std::memset(&a, 0, sizeof a);
  a.mode = VIEW_PLAIN;
  a.a = dy;
  a.ca = L.cinp_t;
  a.B = B;
  a.H = H;
  a.W = W;
  a.cin_p = L.cinp_t;
  a.taps = L.k * L.k;
  a.kp = L.kp_t;
  a.w = net->d_packed_t + L.pkt_off;
  a.bias = net->d_master + L.b_off;  // unused by the data-gradient epilogue
  a.cout = L.cin;
  a.res_scale = 1.0f;
  return a;
}

BwdEpi plain_epi() {
  BwdEpi e;
  std::memset(&e, 0, sizeof e);
  e.mode = EPI_PLAIN;
  e.scale = 1.0f;
  e.stride = NET_FEAT;
  e.out_h_scale = 1.0f;
  return e;
}

namespace {

struct TrainArena {
  uint16_t *xh, *xl, *h0, *fl, *f0h, *rh[NET_NRES + 1], *th[NET_NRES], *U, *g8, *dU, *drh, *dth,
      *df0h, *dflh, *dh0h;
  float *f0f, *rf[2], *out, *dh0a, *dfdf, *drf[2];
};

constexpr int L1_PARTS = 256;

mrs_status ensure_train(mrs_net* net, int B, int H, int W, TrainArena& A) {
  const size_t P = (size_t)B * H * W, p = P / 16;
  std::vector<std::pair<void**, size_t>> plan;
  auto add = [&](void** ptr, size_t bytes) { plan.push_back({ptr, bytes}); };
  add((void**)&A.xh, P * 16 * 2);
  add((void**)&A.xl, p * 8 * 2);
  add((void**)&A.h0, P * 64 * 2);
  add((void**)&A.fl, p * 64 * 2);
  add((void**)&A.f0f, p * 64 * 4);
  add((void**)&A.f0h, p * 64 * 2);
  for (int i = 1; i <= NET_NRES; ++i) add((void**)&A.rh[i], p * 64 * 2);
  for (int i = 0; i < NET_NRES; ++i) add((void**)&A.th[i], p * 64 * 2);
  add((void**)&A.rf[0], p * 64 * 4);
  add((void**)&A.rf[1], p * 64 * 4);
  add((void**)&A.U, p * 256 * 2);
  add((void**)&A.out, P * 3 * 4);
  add((void**)&A.g8, P * 8 * 2);
  add((void**)&A.dU, p * 256 * 2);
  add((void**)&A.dh0a, P * 64 * 4);
  add((void**)&A.dfdf, p * 64 * 4);
  add((void**)&A.drf[0], p * 64 * 4);
  add((void**)&A.drf[1], p * 64 * 4);
  add((void**)&A.drh, p * 64 * 2);
  add((void**)&A.dth, p * 64 * 2);
  add((void**)&A.df0h, p * 64 * 2);
  add((void**)&A.dflh, p * 64 * 2);
  add((void**)&A.dh0h, P * 64 * 2);
  hipStream_t st = current_stream();
  mrs_status rc = arena_carve(net->d_train, net->train_bytes, plan, st, "mrs_train_step");
  if (rc != MRS_OK) return rc;
  A.rh[0] = A.f0h;
  return ensure_wpart(net, (int64_t)P, st);
}

mrs_status ensure_train_state(mrs_net* net) {
  if (net->d_grad) return MRS_OK;
  const size_t n = (size_t)net->nparams;
  if (hipMalloc(&net->d_grad, sizeof(float) * n) != hipSuccess ||
      hipMalloc(&net->d_m, sizeof(float) * n) != hipSuccess ||
      hipMalloc(&net->d_v, sizeof(float) * n) != hipSuccess ||
      hipMalloc(&net->d_packed_t, sizeof(uint16_t) * net->npacked_t) != hipSuccess ||
      hipMalloc(&net->d_loss, sizeof(double)) != hipSuccess ||
      hipMalloc(&net->d_lpart, sizeof(double) * L1_PARTS) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_train_step: optimiser state allocation failed");
  }
  hipStream_t st = current_stream();
  MRS_TRY_HIP(hipMemsetAsync(net->d_m, 0, sizeof(float) * n, st));
  MRS_TRY_HIP(hipMemsetAsync(net->d_v, 0, sizeof(float) * n, st));
  net->adam_step = 0;
  return net_refresh_packed(net, st);
}

// Forward keeping every activation the backward pass reads.
void forward_train(mrs_net* net, const TrainArena& A, int B, int H, int W, const float* hr,
                   const float* aux, const float* lr, hipStream_t st) {
  const std::vector<NetLayer>& Ls = net->layers;
  const int h = H / NET_SCALE, w = W / NET_SCALE;
  const int64_t P = (int64_t)B * H * W, p = P / 16;
  launch_prep(net, P, p, hr, aux, lr, A.xh, A.xl, st);
  ConvArgs a = base_args(net, Ls[0], B, H, W);
  a.a = A.xh;
  a.ca = 16;
  a.relu = 1;
  a.out_h = A.h0;
  a.out_h_stride = NET_FEAT;
  launch_conv(a, Ls[0].cout_p, st);
  a = base_args(net, Ls[1], B, h, w);
  a.a = A.xl;
  a.ca = 8;
  a.relu = 1;
  a.out_h = A.fl;
  a.out_h_stride = NET_FEAT;
  launch_conv(a, Ls[1].cout_p, st);
  a = base_args(net, Ls[2], B, h, w);
  a.mode = VIEW_CONCAT_UNSHUFFLE;
  a.a = A.fl;
  a.ca = NET_FEAT;
  a.b = A.h0;
  a.cb = NET_FEAT;
  a.r = NET_SCALE;
  a.relu = 1;
  a.out_f = A.f0f;
  a.out_f_stride = NET_FEAT;
  a.out_h = A.f0h;
  a.out_h_stride = NET_FEAT;
  launch_conv(a, Ls[2].cout_p, st);
  for (int i = 0; i < NET_NRES; ++i) {
    a = base_args(net, Ls[3 + 2 * i], B, h, w);
    a.a = A.rh[i];
    a.ca = NET_FEAT;
    a.relu = 1;
    a.out_h = A.th[i];
    a.out_h_stride = NET_FEAT;
    launch_conv(a, NET_FEAT, st);
    a = base_args(net, Ls[4 + 2 * i], B, h, w);
    a.a = A.th[i];
    a.ca = NET_FEAT;
    a.res = i == 0 ? A.f0f : A.rf[(i - 1) & 1];
    a.res_scale = NET_RES_SCALE;
    a.res2 = i == NET_NRES - 1 ? A.f0f : nullptr;
    a.out_f = A.rf[i & 1];
    a.out_f_stride = NET_FEAT;
    a.out_h = A.rh[i + 1];
    a.out_h_stride = NET_FEAT;
    launch_conv(a, NET_FEAT, st);
  }
  const NetLayer& Lu = Ls[3 + 2 * NET_NRES];
  const NetLayer& Lr = Ls[4 + 2 * NET_NRES];
  a = base_args(net, Lu, B, h, w);
  a.a = A.rh[NET_NRES];
  a.ca = NET_FEAT;
  a.relu = 1;
  a.out_h = A.U;
  a.out_h_stride = Lu.cout;
  launch_conv(a, Lu.cout_p, st);
  a = base_args(net, Lr, B, H, W);
  a.mode = VIEW_SHUFFLE_CONCAT;
  a.a = A.U;
  a.ca = Lu.cout;
  a.c0 = NET_UPCH;
  a.r = NET_SCALE;
  a.b = A.h0;
  a.cb = NET_FEAT;
  a.out_f = A.out;
  a.out_f_stride = 3;
  launch_conv(a, Lr.cout_p, st);
}

// Backward through the whole network from the BF16 output gradient A.g8;
// writes every layer's gradient into net->d_grad.
void backward(mrs_net* net, const TrainArena& A, int B, int H, int W, hipStream_t st) {
  const std::vector<NetLayer>& Ls = net->layers;
  const int h = H / NET_SCALE, w = W / NET_SCALE;
  const NetLayer& Lu = Ls[3 + 2 * NET_NRES];
  const NetLayer& Lr = Ls[4 + 2 * NET_NRES];
  // rec: d[shuffle(U), h0] -> dU (masked by U > 0, LR layout) and dh0a (FP32)
  {
    ConvArgs a = tconv_args(net, Lr, B, H, W, A.g8);
    BwdEpi e = plain_epi();
    e.mode = EPI_REC_SPLIT;
    e.stride = NET_FEAT;
    e.out_f = A.dh0a;
    e.out_h = A.dU;
    e.mask = A.U;
    e.c_split = NET_UPCH;
    e.stride2 = Lu.cout;
    e.r = NET_SCALE;
    launch_dgrad(a, e, Lr.coutp_t, st);
    ConvArgs x = base_args(net, Lr, B, H, W);
    x.mode = VIEW_SHUFFLE_CONCAT;
    x.a = A.U;
    x.ca = Lu.cout;
    x.c0 = NET_UPCH;
    x.r = NET_SCALE;
    x.b = A.h0;
    x.cb = NET_FEAT;
    wgrad(net, Lr, x, A.g8, 8, st);
  }
  // up: dFDF (FP32) and 0.1 dFDF (BF16) = gradient of the last trunk conv
  {
    ConvArgs a = tconv_args(net, Lu, B, h, w, A.dU);
    BwdEpi e = plain_epi();
    e.out_f = A.dfdf;
    e.out_h = A.drh;
    e.out_h_scale = NET_RES_SCALE;
    launch_dgrad(a, e, Lu.coutp_t, st);
    ConvArgs x = base_args(net, Lu, B, h, w);
    x.a = A.rh[NET_NRES];
    x.ca = NET_FEAT;
    wgrad(net, Lu, x, A.dU, Lu.cout, st);
  }
  const float* dr = A.dfdf;
  for (int i = NET_NRES - 1; i >= 0; --i) {
    const NetLayer& La = Ls[3 + 2 * i];
    const NetLayer& Lb = Ls[4 + 2 * i];
    {  // conv b: dt = (W_b^T * 0.1 dr) masked by t > 0
      ConvArgs a = tconv_args(net, Lb, B, h, w, A.drh);
      BwdEpi e = plain_epi();
      e.mask = A.th[i];
      e.out_h = A.dth;
      launch_dgrad(a, e, Lb.coutp_t, st);
      ConvArgs x = base_args(net, Lb, B, h, w);
      x.a = A.th[i];
      x.ca = NET_FEAT;
      wgrad(net, Lb, x, A.drh, NET_FEAT, st);
    }
    {  // conv a: dr_i = dr_{i+1} + W_a^T dt; at i = 0 add dFDF and mask by F0 > 0
      ConvArgs a = tconv_args(net, La, B, h, w, A.dth);
      BwdEpi e = plain_epi();
      e.add1 = dr;
      if (i > 0) {
        e.out_f = A.drf[i & 1];
        e.out_h = A.drh;
        e.out_h_scale = NET_RES_SCALE;
      } else {
        e.add2 = A.dfdf;
        e.mask = A.f0h;
        e.out_h = A.df0h;
      }
      launch_dgrad(a, e, La.coutp_t, st);
      ConvArgs x = base_args(net, La, B, h, w);
      x.a = A.rh[i];
      x.ca = NET_FEAT;
      wgrad(net, La, x, A.dth, NET_FEAT, st);
      dr = A.drf[i & 1];
    }
  }
  // fuse: d[fl, unshuffle(h0)] -> dfl (masked) and dh0 = (dh0a + shuffle(.)) masked
  {
    const NetLayer& Lf = Ls[2];
    ConvArgs a = tconv_args(net, Lf, B, h, w, A.df0h);
    BwdEpi e = plain_epi();
    e.mode = EPI_FUSE_SPLIT;
    e.c_split = NET_FEAT;
    e.stride = NET_FEAT;
    e.mask = A.fl;
    e.out_h = A.dflh;
    e.add1 = A.dh0a;
    e.mask2 = A.h0;
    e.out_h2 = A.dh0h;
    e.r = NET_SCALE;
    launch_dgrad(a, e, Lf.coutp_t, st);
    ConvArgs x = base_args(net, Lf, B, h, w);
    x.mode = VIEW_CONCAT_UNSHUFFLE;
    x.a = A.fl;
    x.ca = NET_FEAT;
    x.b = A.h0;
    x.cb = NET_FEAT;
    x.r = NET_SCALE;
    wgrad(net, Lf, x, A.df0h, NET_FEAT, st);
  }
  {  // encoders: weight gradients only
    ConvArgs x = base_args(net, Ls[1], B, h, w);
    x.a = A.xl;
    x.ca = 8;
    wgrad(net, Ls[1], x, A.dflh, NET_FEAT, st);
    x = base_args(net, Ls[0], B, H, W);
    x.a = A.xh;
    x.ca = 16;
    wgrad(net, Ls[0], x, A.dh0h, NET_FEAT, st);
  }
}

mrs_status check_train_args(mrs_net* n, int B, const float* hr, const float* aux,
                            const float* lr, const float* tgt, int W, int H) {
  if (!n) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_train_step: net is NULL");
  if (!hr || !aux || !lr || !tgt)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_train_step: NULL buffer");
  const int sc = arch_scale(n->arch);
  if (B < 1 || W < sc || H < sc || W % sc || H % sc || (int64_t)B * W * H > (int64_t)1 << 26)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_train_step: W, H multiples of the net's scale (" + std::to_string(sc) +
                    "), B >= 1, B*W*H <= 2^26");
  if (((uintptr_t)hr | (uintptr_t)aux | (uintptr_t)lr | (uintptr_t)tgt) & 3u)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_train_step: buffers must be 4-byte aligned");
  if (!n->has_params) return fail(MRS_ERR_NOT_READY, "mrs_train_step: no parameters");
  if (arch_has_layers(n->arch) && !n->in_layers)
    return fail(MRS_ERR_NOT_READY, "mrs_train_step: bind the HRLS render layers first "
                                   "(mrs_net_bind_layers)");
  return MRS_OK;
}

// Forward, output gradient (a loss against tgt, or the caller's gout when tgt
// is NULL) and backward into n->d_grad; *out = the network output.
mrs_status loss_and_grad(mrs_net* n, int B, const float* hr, const float* aux, const float* lr,
                         const float* tgt, const float* gout, int W, int H, float beta,
                         hipStream_t st, const float** out) {
  mrs_status rc = ensure_train_state(n);
  if (rc != MRS_OK) return rc;
  OutGrad og;
  og.tgt = tgt;
  og.beta = beta;
  og.gout = gout;
  og.part = n->d_lpart;
  og.nparts = L1_PARTS;
  og.loss = n->d_loss;
  if (arch_is_rdg(n->arch)) return rdg_loss_grad(n, B, H, W, hr, aux, lr, og, out, st);
  TrainArena A;
  rc = ensure_train(n, B, H, W, A);
  if (rc != MRS_OK) return rc;
  prof_begin(KID_TRAIN_FWD, st);
  forward_train(n, A, B, H, W, hr, aux, lr, st);
  prof_end(KID_TRAIN_FWD, st);
  launch_out_grad(og, A.out, (int64_t)B * H * W, A.g8, st);
  prof_begin(KID_TRAIN_BWD, st);
  backward(n, A, B, H, W, st);
  prof_end(KID_TRAIN_BWD, st);
  MRS_TRY_HIP(hipGetLastError());
  *out = A.out;
  return MRS_OK;
}

int64_t arch_params(int32_t arch) {
  if (arch == MRS_NET_RES16) return NET_NUM_PARAMS;
  if (!arch_known(arch)) return -1;
  int64_t n = 0;
  for (const NetLayer& L : make_layers(arch)) n += (int64_t)L.cout * L.cin * L.k * L.k + L.cout;
  return n;
}

mrs_status check_loss(int32_t loss, float beta, const char* who) {
  if (loss != MRS_LOSS_L1 && loss != MRS_LOSS_ROBUST)
    return fail(MRS_ERR_INVALID_ARGUMENT, std::string(who) + ": unknown loss");
  if (loss == MRS_LOSS_ROBUST && !(beta > 0.0f && std::isfinite(beta)))
    return fail(MRS_ERR_INVALID_ARGUMENT, std::string(who) + ": the robust loss needs beta > 0");
  return MRS_OK;
}

}  // namespace

}  // namespace mrs

using namespace mrs;

extern "C" {

int64_t mrs_net_num_params(void) { return NET_NUM_PARAMS; }

int64_t mrs_net_arch_num_params(int32_t arch) { return arch_params(arch); }

mrs_status mrs_net_create_arch(int32_t arch, mrs_net** out) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_create: out is NULL");
  *out = nullptr;
  if (arch_params(arch) < 0) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_create: unknown arch");
  mrs_net* n = new mrs_net();
  n->arch = arch;
  n->layers = make_layers(arch);
  const NetLayer& last = n->layers.back();
  n->nparams = last.b_off + last.cout;
  n->npacked = last.pk_off + (int64_t)last.cout_p * last.kp;
  n->npacked_t = 0;
  for (const NetLayer& L : n->layers)
    if (L.pkt_off >= 0) n->npacked_t = std::max(n->npacked_t, L.pkt_off + (int64_t)L.coutp_t * L.kp_t);
  if (n->nparams != arch_params(arch)) {
    delete n;
    return fail(MRS_ERR_DEVICE, "mrs_net_create: internal layer table mismatch");
  }
  if (hipMalloc(&n->d_master, sizeof(float) * n->nparams) != hipSuccess ||
      hipMalloc(&n->d_packed, sizeof(uint16_t) * n->npacked) != hipSuccess) {
    (void)hipGetLastError();
    if (n->d_master) (void)hipFree(n->d_master);
    delete n;
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_net_create: parameter allocation failed");
  }
  *out = n;
  return MRS_OK;
}

mrs_status mrs_net_create(mrs_net** out) { return mrs_net_create_arch(MRS_NET_RES16, out); }

mrs_status mrs_net_bind_layers(mrs_net* n, const float* layers_dev, const float* sumsq_dev,
                               int32_t spp) {
  if (!n) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_bind_layers: net is NULL");
  if (!arch_has_layers(n->arch))
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_net_bind_layers: this architecture takes no render layers");
  if (!layers_dev && !sumsq_dev && spp == 0) {  // unbind
    n->in_layers = n->in_sumsq = nullptr;
    n->in_spp = 0;
    return MRS_OK;
  }
  if (!layers_dev || !sumsq_dev || spp < 1 || (((uintptr_t)layers_dev | (uintptr_t)sumsq_dev) & 3u))
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_net_bind_layers: layers and sums of squares must be non-NULL, 4-byte "
                "aligned device buffers and spp >= 1");
  n->in_layers = layers_dev;
  n->in_sumsq = sumsq_dev;
  n->in_spp = spp;
  return MRS_OK;
}

mrs_status mrs_net_destroy(mrs_net* n) {
  if (!n) return MRS_OK;
  (void)hipDeviceSynchronize();
  if (n->d_master) (void)hipFree(n->d_master);
  if (n->d_packed) (void)hipFree(n->d_packed);
  if (n->d_arena) (void)hipFree(n->d_arena);
  for (void* p : {(void*)n->d_packed_t, (void*)n->d_grad, (void*)n->d_m, (void*)n->d_v,
                  (void*)n->d_train, (void*)n->d_loss, (void*)n->d_lpart, (void*)n->d_wpart,
                  (void*)n->d_bpart, (void*)n->d_packjobs})
    if (p) (void)hipFree(p);
  delete n;
  return MRS_OK;
}

mrs_status mrs_net_init(mrs_net* n, uint64_t seed) {
  if (!n) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_init: net is NULL");
  hipStream_t st = current_stream();
  for (const NetLayer& L : n->layers) launch_init(n->d_master + L.w_off, L, seed, st);
  mrs_status rc = net_refresh_packed(n, st);
  if (rc != MRS_OK) return rc;
  n->has_params = true;
  return MRS_OK;
}

mrs_status mrs_net_set_params(mrs_net* n, const float* params, int64_t count) {
  if (!n || !params) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_set_params: NULL argument");
  if (count != n->nparams)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_set_params: expected " +
                                              std::to_string(n->nparams) + " parameters");
  hipStream_t st = current_stream();
  MRS_TRY_HIP(hipMemcpyAsync(n->d_master, params, sizeof(float) * count, hipMemcpyHostToDevice, st));
  mrs_status rc = net_refresh_packed(n, st);
  if (rc != MRS_OK) return rc;
  MRS_TRY_HIP(hipStreamSynchronize(st));
  n->has_params = true;
  return MRS_OK;
}

mrs_status mrs_net_get_params(const mrs_net* n, float* params, int64_t count) {
  if (!n || !params) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_get_params: NULL argument");
  if (count != n->nparams)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_get_params: wrong count");
  if (!n->has_params) return fail(MRS_ERR_NOT_READY, "mrs_net_get_params: no parameters");
  hipStream_t st = current_stream();
  MRS_TRY_HIP(hipMemcpyAsync(params, n->d_master, sizeof(float) * count, hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  return MRS_OK;
}

mrs_status mrs_fuse_batch(mrs_net* n, int32_t B, const float* hr, const float* aux,
                          const float* lr, int32_t W, int32_t H, float* out) {
  if (!n) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_fuse: net is NULL");
  if (!hr || !aux || !lr || !out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_fuse: NULL buffer");
  const int sc = arch_scale(n->arch);
  if (B < 1 || W < sc || H < sc || W % sc || H % sc || W > 16384 || H > 16384 ||
      (int64_t)B * W * H > (int64_t)1 << 30)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_fuse: W and H must be multiples of the net's scale (" + std::to_string(sc) +
                    ") in [scale, 16384], B >= 1, B*W*H <= 2^30");
  if (((uintptr_t)hr | (uintptr_t)aux | (uintptr_t)lr | (uintptr_t)out) & 3u)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_fuse: buffers must be 4-byte aligned");
  if (!n->has_params) return fail(MRS_ERR_NOT_READY, "mrs_fuse: no network parameters loaded");
  if (arch_has_layers(n->arch) && !n->in_layers)
    return fail(MRS_ERR_NOT_READY, "mrs_fuse: bind the HRLS render layers first "
                                   "(mrs_net_bind_layers)");
  if (arch_is_rdg(n->arch)) return rdg_forward(n, B, H, W, hr, aux, lr, out, current_stream());
  return net_forward(n, B, H, W, hr, aux, lr, out, current_stream());
}

mrs_status mrs_fuse(mrs_net* n, const float* hr, const float* aux, const float* lr, int32_t W,
                    int32_t H, float* out) {
  return mrs_fuse_batch(n, 1, hr, aux, lr, W, H, out);
}

mrs_status mrs_net_loss_grad_ex(mrs_net* n, int32_t B, const float* hr, const float* aux,
                                const float* lr, const float* tgt, int32_t W, int32_t H,
                                int32_t loss, float beta, float* grad_host, double* loss_host,
                                float* out_dev) {
  mrs_status rc = check_train_args(n, B, hr, aux, lr, tgt, W, H);
  if (rc != MRS_OK) return rc;
  rc = check_loss(loss, beta, "mrs_net_loss_grad");
  if (rc != MRS_OK) return rc;
  hipStream_t st = current_stream();
  const float* out = nullptr;
  rc = loss_and_grad(n, B, hr, aux, lr, tgt, nullptr, W, H, loss == MRS_LOSS_ROBUST ? beta : 0.0f,
                     st, &out);
  if (rc != MRS_OK) return rc;
  if (out_dev)
    MRS_TRY_HIP(hipMemcpyAsync(out_dev, out, sizeof(float) * 3 * (size_t)B * H * W,
                               hipMemcpyDeviceToDevice, st));
  if (grad_host)
    MRS_TRY_HIP(hipMemcpyAsync(grad_host, n->d_grad, sizeof(float) * n->nparams,
                               hipMemcpyDeviceToHost, st));
  if (loss_host) MRS_TRY_HIP(hipMemcpyAsync(loss_host, n->d_loss, sizeof(double), hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  return MRS_OK;
}

mrs_status mrs_net_backward(mrs_net* n, int32_t B, const float* hr, const float* aux,
                            const float* lr, int32_t W, int32_t H, const float* grad_out_dev,
                            float* grad_host) {
  mrs_status rc = check_train_args(n, B, hr, aux, lr, grad_out_dev, W, H);
  if (rc != MRS_OK) return rc;
  hipStream_t st = current_stream();
  const float* out = nullptr;
  rc = loss_and_grad(n, B, hr, aux, lr, nullptr, grad_out_dev, W, H, 0.0f, st, &out);
  if (rc != MRS_OK) return rc;
  if (grad_host)
    MRS_TRY_HIP(hipMemcpyAsync(grad_host, n->d_grad, sizeof(float) * n->nparams,
                               hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  return MRS_OK;
}

mrs_status mrs_net_loss_grad(mrs_net* n, int32_t B, const float* hr, const float* aux,
                             const float* lr, const float* tgt, int32_t W, int32_t H,
                             float* grad_host, double* loss_host, float* out_dev) {
  return mrs_net_loss_grad_ex(n, B, hr, aux, lr, tgt, W, H, MRS_LOSS_L1, 0.0f, grad_host,
                              loss_host, out_dev);
}

mrs_status mrs_train_step_ex(mrs_net* n, int32_t B, const float* hr, const float* aux,
                             const float* lr, const float* tgt, int32_t W, int32_t H,
                             const mrs_train_opts* opts, double* loss_host) {
  mrs_status rc = check_train_args(n, B, hr, aux, lr, tgt, W, H);
  if (rc != MRS_OK) return rc;
  if (!opts) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_train_step: opts is NULL");
  rc = check_loss(opts->loss, opts->beta, "mrs_train_step");
  if (rc != MRS_OK) return rc;
  if (opts->optimizer != MRS_OPT_ADAM && opts->optimizer != MRS_OPT_SGD)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_train_step: unknown optimizer");
  if (!(opts->lr > 0.0f) || !std::isfinite(opts->lr))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_train_step: learning rate must be positive");
  hipStream_t st = current_stream();
  const float* out = nullptr;
  rc = loss_and_grad(n, B, hr, aux, lr, tgt, nullptr, W, H,
                     opts->loss == MRS_LOSS_ROBUST ? opts->beta : 0.0f, st, &out);
  if (rc != MRS_OK) return rc;
  prof_begin(KID_TRAIN_ADAM, st);
  if (opts->optimizer == MRS_OPT_ADAM) {
    n->adam_step += 1;
    const double t = (double)n->adam_step;
    const float c1 = (float)(1.0 - std::pow(0.9, t)), c2 = (float)(1.0 - std::pow(0.999, t));
    launch_adam(n->d_master, n->d_grad, n->d_m, n->d_v, n->nparams, opts->lr, 0.9f, 0.999f,
                1e-8f, c1, c2, st);
  } else {
    launch_sgd(n->d_master, n->d_grad, n->nparams, opts->lr, st);
  }
  rc = net_refresh_packed(n, st);
  prof_end(KID_TRAIN_ADAM, st);
  if (rc != MRS_OK) return rc;
  if (loss_host) {
    MRS_TRY_HIP(hipMemcpyAsync(loss_host, n->d_loss, sizeof(double), hipMemcpyDeviceToHost, st));
    MRS_TRY_HIP(hipStreamSynchronize(st));
  }
  return MRS_OK;
}

mrs_status mrs_train_step(mrs_net* n, int32_t B, const float* hr, const float* aux,
                          const float* lr, const float* tgt, int32_t W, int32_t H, float lr_rate,
                          double* loss_host) {
  mrs_train_opts o;
  o.loss = MRS_LOSS_L1;
  o.beta = 0.0f;
  o.optimizer = MRS_OPT_ADAM;
  o.lr = lr_rate;
  return mrs_train_step_ex(n, B, hr, aux, lr, tgt, W, H, &o, loss_host);
}

mrs_status mrs_net_get_state(const mrs_net* n, float* params, float* m, float* v, int64_t count,
                             int64_t* step) {
  if (!n || !params || !m || !v || !step || count != n->nparams)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_get_state: bad arguments");
  if (!n->has_params) return fail(MRS_ERR_NOT_READY, "mrs_net_get_state: no parameters");
  hipStream_t st = current_stream();
  const size_t b = sizeof(float) * count;
  MRS_TRY_HIP(hipMemcpyAsync(params, n->d_master, b, hipMemcpyDeviceToHost, st));
  if (n->d_m) {
    MRS_TRY_HIP(hipMemcpyAsync(m, n->d_m, b, hipMemcpyDeviceToHost, st));
    MRS_TRY_HIP(hipMemcpyAsync(v, n->d_v, b, hipMemcpyDeviceToHost, st));
  } else {
    std::memset(m, 0, b);
    std::memset(v, 0, b);
  }
  MRS_TRY_HIP(hipStreamSynchronize(st));
  *step = n->adam_step;
  return MRS_OK;
}

mrs_status mrs_net_set_state(mrs_net* n, const float* params, const float* m, const float* v,
                             int64_t count, int64_t step) {
  if (!n || !params || !m || !v || count != n->nparams || step < 0)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_set_state: bad arguments");
  hipStream_t st = current_stream();
  MRS_TRY_HIP(hipMemcpyAsync(n->d_master, params, sizeof(float) * count, hipMemcpyHostToDevice, st));
  n->has_params = true;
  mrs_status rc = ensure_train_state(n);
  if (rc != MRS_OK) return rc;
  MRS_TRY_HIP(hipMemcpyAsync(n->d_m, m, sizeof(float) * count, hipMemcpyHostToDevice, st));
  MRS_TRY_HIP(hipMemcpyAsync(n->d_v, v, sizeof(float) * count, hipMemcpyHostToDevice, st));
  n->adam_step = step;
  rc = net_refresh_packed(n, st);
  if (rc != MRS_OK) return rc;
  MRS_TRY_HIP(hipStreamSynchronize(st));
  return MRS_OK;
}

}  // extern "C"

namespace {

// CRC-32 of IEEE 802.3 (reflected polynomial 0xEDB88320), table driven.
uint32_t crc32_update(uint32_t crc, const void* data, size_t n) {
  static uint32_t table[256];
  static bool ready = [] {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      table[i] = c;
    }
    return true;
  }();
  (void)ready;
  const uint8_t* p = static_cast<const uint8_t*>(data);
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xffu] ^ (crc >> 8);
  return ~crc;
}

// Checkpoint file layout (little-endian), 48-byte header then the body:
//   char magic[8] "MRSCKPT\0", u32 version (1), i32 arch, i64 count,
//   i64 Adam step, u64 data counter, u32 CRC-32 of the body, u32 CRC-32 of
//   the 44 header bytes before it; body = count FP32 masters, count Adam m,
//   count Adam v.
constexpr char CKPT_MAGIC[8] = {'M', 'R', 'S', 'C', 'K', 'P', 'T', '\0'};
constexpr uint32_t CKPT_VERSION = 1;
struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t arch;
  int64_t count;
  int64_t step;
  uint64_t data_counter;
  uint32_t body_crc;
  uint32_t header_crc;
};
static_assert(sizeof(CkptHeader) == 48, "checkpoint header layout");

}  // namespace

extern "C" {

mrs_status mrs_net_save(const mrs_net* n, const char* path, uint64_t data_counter) {
  if (!n || !path) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_save: NULL argument");
  if (!n->has_params) return fail(MRS_ERR_NOT_READY, "mrs_net_save: no parameters");
  const int64_t cnt = n->nparams;
  std::vector<float> body(3 * (size_t)cnt);
  int64_t step = 0;
  mrs_status rc = mrs_net_get_state(n, body.data(), body.data() + cnt, body.data() + 2 * cnt, cnt,
                                    &step);
  if (rc != MRS_OK) return rc;
  CkptHeader h;
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.version = CKPT_VERSION;
  h.arch = n->arch;
  h.count = cnt;
  h.step = step;
  h.data_counter = data_counter;
  h.body_crc = crc32_update(0u, body.data(), sizeof(float) * body.size());
  h.header_crc = crc32_update(0u, &h, offsetof(CkptHeader, header_crc));
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_save: cannot open " + tmp);
  const bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 &&
                  std::fwrite(body.data(), sizeof(float), body.size(), f) == body.size();
  if (std::fclose(f) != 0 || !ok) {
    std::remove(tmp.c_str());
    return fail(MRS_ERR_DEVICE, "mrs_net_save: write to " + tmp + " failed");
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(MRS_ERR_DEVICE, std::string("mrs_net_save: cannot rename to ") + path);
  }
  return MRS_OK;
}

mrs_status mrs_net_load(mrs_net* n, const char* path, uint64_t* data_counter) {
  if (!n || !path) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_load: NULL argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(MRS_ERR_INVALID_ARGUMENT, std::string("mrs_net_load: cannot open ") + path);
  CkptHeader h;
  std::vector<float> body;
  std::string err;
  if (std::fread(&h, sizeof h, 1, f) != 1 || std::memcmp(h.magic, CKPT_MAGIC, 8) != 0) {
    err = "not a checkpoint file";
  } else if (h.header_crc != crc32_update(0u, &h, offsetof(CkptHeader, header_crc))) {
    err = "header checksum mismatch";
  } else if (h.version != CKPT_VERSION) {
    err = "unsupported checkpoint version " + std::to_string(h.version);
  } else if (h.arch != n->arch || h.count != n->nparams) {
    err = "checkpoint of another network (arch " + std::to_string(h.arch) + ", " +
          std::to_string(h.count) + " parameters)";
  } else if (h.step < 0) {
    err = "negative step";
  } else {
    body.resize(3 * (size_t)h.count);
    char extra;
    if (std::fread(body.data(), sizeof(float), body.size(), f) != body.size() ||
        std::fread(&extra, 1, 1, f) != 0)
      err = "truncated or oversized file";
    else if (h.body_crc != crc32_update(0u, body.data(), sizeof(float) * body.size()))
      err = "body checksum mismatch";
  }
  std::fclose(f);
  if (!err.empty()) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_load: " + err);
  const int64_t cnt = h.count;
  mrs_status rc = mrs_net_set_state(n, body.data(), body.data() + cnt, body.data() + 2 * cnt, cnt,
                                    h.step);
  if (rc != MRS_OK) return rc;
  if (data_counter) *data_counter = h.data_counter;
  return MRS_OK;
}

mrs_status mrs_debug_net_activation(const mrs_net* n, int32_t which, float* out_host,
                                    int64_t count) {
  if (!n || !out_host) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_net_activation: NULL");
  if (!n->last_f0) return fail(MRS_ERR_NOT_READY, "mrs_debug_net_activation: no forward yet");
  const int sc = arch_scale(n->arch);
  const int64_t want = (int64_t)n->last_B * (n->last_H / sc) * (n->last_W / sc) * NET_FEAT;
  if (count != want || (which != 0 && which != 1))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_net_activation: bad which/count");
  hipStream_t st = current_stream();
  MRS_TRY_HIP(hipMemcpyAsync(out_host, which == 0 ? n->last_f0 : n->last_fdf,
                             sizeof(float) * count, hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  return MRS_OK;
}

}  // extern "C"
