// Host side of the fusion network: layer table, parameters, forward pass.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "mrs_internal.hpp"
#include "cnn.hpp"

namespace mrs {
namespace {

int round_up(int v, int m) { return (v + m - 1) / m * m; }

std::vector<NetLayer> make_layers() {
  struct S {
    const char* name;
    int cout, cin, k, cin_p;
  };
  static std::vector<std::string> names;
  std::vector<S> specs = {{"hrls", NET_FEAT, 10, 3, 16},
                          {"lrhs", NET_FEAT, 3, 3, 8},
                          {"fuse", NET_FEAT, NET_FEAT + NET_SCALE * NET_SCALE * NET_FEAT, 1,
                           NET_FEAT + NET_SCALE * NET_SCALE * NET_FEAT}};
  if (names.empty()) {
    for (int i = 0; i < NET_NRES; ++i) {
      names.push_back("res" + std::to_string(i) + "a");
      names.push_back("res" + std::to_string(i) + "b");
    }
  }
  for (int i = 0; i < 2 * NET_NRES; ++i) specs.push_back({names[i].c_str(), NET_FEAT, NET_FEAT, 3, NET_FEAT});
  specs.push_back({"up", NET_UPCH * NET_SCALE * NET_SCALE, NET_FEAT, 3, NET_FEAT});
  specs.push_back({"rec", 3, NET_UPCH + NET_FEAT, 3, NET_UPCH + NET_FEAT});
  std::vector<NetLayer> L;
  int64_t off = 0, pk = 0;
  for (const S& s : specs) {
    NetLayer l;
    l.name = s.name;
    l.cout = s.cout;
    l.cin = s.cin;
    l.k = s.k;
    l.cin_p = s.cin_p;
    l.kp = round_up(s.k * s.k * s.cin_p, 32);
    l.cout_p = s.cout >= 64 ? round_up(s.cout, 64) : round_up(s.cout, 16);
    l.w_off = off;
    off += (int64_t)s.cout * s.cin * s.k * s.k;
    l.b_off = off;
    off += s.cout;
    l.pk_off = pk;
    pk += (int64_t)l.cout_p * l.kp;
    L.push_back(l);
  }
  return L;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Arena {
  uint16_t *xh, *xl, *h0, *fl, *f0h, *rh[2], *th, *U;
  float *f0f, *rf[2];
};

mrs_status ensure_arena(mrs_net* net, int B, int H, int W, Arena& A) {
  const size_t P = (size_t)B * H * W, p = P / 16;
  size_t off = 0;
  size_t o_xh = off; off += align256(P * 16 * 2);
  size_t o_xl = off; off += align256(p * 8 * 2);
  size_t o_h0 = off; off += align256(P * 64 * 2);
  size_t o_fl = off; off += align256(p * 64 * 2);
  size_t o_f0f = off; off += align256(p * 64 * 4);
  size_t o_f0h = off; off += align256(p * 64 * 2);
  size_t o_rf0 = off; off += align256(p * 64 * 4);
  size_t o_rf1 = off; off += align256(p * 64 * 4);
  size_t o_rh0 = off; off += align256(p * 64 * 2);
  size_t o_rh1 = off; off += align256(p * 64 * 2);
  size_t o_th = off; off += align256(p * 64 * 2);
  size_t o_U = off; off += align256(p * 256 * 2);
  if (off > net->arena_bytes) {
    if (net->d_arena) {
      MRS_TRY_HIP(hipStreamSynchronize(current_stream()));
      (void)hipFree(net->d_arena);
    }
    net->d_arena = nullptr;
    net->arena_bytes = 0;
    if (hipMalloc(&net->d_arena, off) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_fuse: activation allocation failed");
    }
    net->arena_bytes = off;
  }
  char* b = net->d_arena;
  A.xh = (uint16_t*)(b + o_xh);
  A.xl = (uint16_t*)(b + o_xl);
  A.h0 = (uint16_t*)(b + o_h0);
  A.fl = (uint16_t*)(b + o_fl);
  A.f0f = (float*)(b + o_f0f);
  A.f0h = (uint16_t*)(b + o_f0h);
  A.rf[0] = (float*)(b + o_rf0);
  A.rf[1] = (float*)(b + o_rf1);
  A.rh[0] = (uint16_t*)(b + o_rh0);
  A.rh[1] = (uint16_t*)(b + o_rh1);
  A.th = (uint16_t*)(b + o_th);
  A.U = (uint16_t*)(b + o_U);
  return MRS_OK;
}

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

}  // namespace

mrs_status net_forward(mrs_net* net, int B, int H, int W, const float* hr, const float* aux,
                       const float* lr, float* out, hipStream_t st) {
  Arena A;
  mrs_status rc = ensure_arena(net, B, H, W, A);
  if (rc != MRS_OK) return rc;
  const std::vector<NetLayer>& Ls = net->layers;
  const int h = H / NET_SCALE, w = W / NET_SCALE;
  const int64_t P = (int64_t)B * H * W, p = P / 16;
  prof_begin(KID_CNN_PREP, st);
  launch_prep(P, p, hr, aux, lr, A.xh, A.xl, st);
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
    launch_conv(a, La.cout_p, st);
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
    launch_conv(bb, Lb.cout_p, st);
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

mrs_status net_refresh_packed(mrs_net* net, hipStream_t st) {
  for (const NetLayer& L : net->layers)
    launch_pack(net->d_master + L.w_off, L, net->d_packed + L.pk_off, st);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

}  // namespace mrs

using namespace mrs;

extern "C" {

int64_t mrs_net_num_params(void) { return NET_NUM_PARAMS; }

mrs_status mrs_net_create(mrs_net** out) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_net_create: out is NULL");
  *out = nullptr;
  mrs_net* n = new mrs_net();
  n->layers = make_layers();
  const NetLayer& last = n->layers.back();
  n->nparams = last.b_off + last.cout;
  n->npacked = last.pk_off + (int64_t)last.cout_p * last.kp;
  if (n->nparams != NET_NUM_PARAMS) {
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

mrs_status mrs_net_destroy(mrs_net* n) {
  if (!n) return MRS_OK;
  (void)hipDeviceSynchronize();
  if (n->d_master) (void)hipFree(n->d_master);
  if (n->d_packed) (void)hipFree(n->d_packed);
  if (n->d_arena) (void)hipFree(n->d_arena);
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
  if (B < 1 || W < 4 || H < 4 || W % 4 || H % 4 || W > 16384 || H > 16384 ||
      (int64_t)B * W * H > (int64_t)1 << 30)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_fuse: W and H must be multiples of 4 in [4, 16384], B >= 1, B*W*H <= 2^30");
  if (((uintptr_t)hr | (uintptr_t)aux | (uintptr_t)lr | (uintptr_t)out) & 3u)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_fuse: buffers must be 4-byte aligned");
  if (!n->has_params) return fail(MRS_ERR_NOT_READY, "mrs_fuse: no network parameters loaded");
  return net_forward(n, B, H, W, hr, aux, lr, out, current_stream());
}

mrs_status mrs_fuse(mrs_net* n, const float* hr, const float* aux, const float* lr, int32_t W,
                    int32_t H, float* out) {
  return mrs_fuse_batch(n, 1, hr, aux, lr, W, H, out);
}

mrs_status mrs_debug_net_activation(const mrs_net* n, int32_t which, float* out_host,
                                    int64_t count) {
  if (!n || !out_host) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_net_activation: NULL");
  if (!n->last_f0) return fail(MRS_ERR_NOT_READY, "mrs_debug_net_activation: no forward yet");
  const int64_t want = (int64_t)n->last_B * (n->last_H / 4) * (n->last_W / 4) * NET_FEAT;
  if (count != want || (which != 0 && which != 1))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_net_activation: bad which/count");
  hipStream_t st = current_stream();
  MRS_TRY_HIP(hipMemcpyAsync(out_host, which == 0 ? n->last_f0 : n->last_fdf,
                             sizeof(float) * count, hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  return MRS_OK;
}

}  // extern "C"
