// Fusion network of the hybrid method on gfx950: every convolution is an
// implicit GEMM on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; the residual stream stays FP32; weights keep FP32 masters and
// BF16 packed copies.
//
// Architecture (paper Sec. 4; trunk of 16 residual blocks):
//   h0  = ReLU(conv3x3 10->64 (HRLS rgb + albedo + normal + depth))   @HR
//   fl  = ReLU(conv3x3 3->64  (LRHS rgb))                              @LR
//   F0  = ReLU(conv1x1 [fl, unshuffle4(h0)] 1088->64)                 @LR
//   r   <- r + 0.1 conv3x3(ReLU(conv3x3(r))), 16 times, r_0 = F0      @LR
//   FDF = r_16 + F0
//   U   = ReLU(conv3x3 64->256 (FDF))                                  @LR
//   out = conv3x3 [shuffle4(U), h0] 80->3                              @HR
// The (un)shuffles are never materialised: they are folded into the input
// addressing of the convs that read them.  Channel conventions: unshuffle by r
// puts HR pixel (rY+i, rX+j) channel c at LR channel (i r + j) C + c; shuffle
// is its inverse.
//
// GEMM mapping: M = output pixels (NHWC raster order), N = output channels,
// K = taps x padded input channels.  A wave computes 32 pixels x (16 NT)
// channels: 2 x NT accumulator tiles of 16x16.  Per 32-wide K step, lane l
// loads the 8 consecutive input channels (one 16-byte load) of pixel l%16 of
// each row tile for K chunk l/16, and the matching 8 weights of output channel
// l%16 of each column tile.
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mrs_internal.hpp"
#include "devmath.hpp"
#include "cnn.hpp"

namespace mrs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 zero8() {
  uint4 z = make_uint4(0u, 0u, 0u, 0u);
  return __builtin_bit_cast(bf16x8, z);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

// Offset (I, J) inside its r x r block of the HR pixel held by unshuffle slot
// q.  One stride-r unshuffle (dsf = 0): q = I r + J.  dsf stacked stride-2
// deshuffles (r = 2^dsf), the first consuming the low bits: base-4 digit k of
// q is 2 (bit k of I) + (bit k of J).
__device__ __forceinline__ void unshuffle_slot(int q, int r, int dsf, int& I, int& J) {
  if (dsf) {
    I = J = 0;
    for (int k = 0; k < dsf; ++k) {
      J |= ((q >> (2 * k)) & 1) << k;
      I |= ((q >> (2 * k + 1)) & 1) << k;
    }
  } else {
    I = q / r;
    J = q - I * r;
  }
}

// Address of channel c of the conv input at pixel (b, y, x) through the view
// (nullptr outside the image); channels c .. c+7 are contiguous there when c is
// a multiple of 8.
__device__ __forceinline__ const uint16_t* view_ptr(const ConvArgs& p, int b, int y, int x,
                                                    int c) {
  if (y < 0 || y >= p.H || x < 0 || x >= p.W) return nullptr;
  switch (p.mode) {
    case VIEW_PLAIN:
      return p.a + ((size_t)(b * p.H + y) * p.W + x) * p.ca + c;
    case VIEW_CONCAT_UNSHUFFLE:  // [a (LR, ca ch), unshuffle_r(b (HR, cb ch))]
      if (c < p.ca) {
        return p.a + ((size_t)(b * p.H + y) * p.W + x) * p.ca + c;
      } else {
        const int cc = c - p.ca;
        const int qq = cc / p.cb, ch = cc - qq * p.cb;
        int I, J;
        unshuffle_slot(qq, p.r, p.dsf, I, J);
        const int hy = y * p.r + I, hx = x * p.r + J;
        return p.b + ((size_t)(b * p.H * p.r + hy) * (p.W * p.r) + hx) * p.cb + ch;
      }
    default:  // VIEW_SHUFFLE_CONCAT: [shuffle_r(a (LR, ca = r^2 c0 ch)), b (HR, cb ch)]
      if (c < p.c0) {
        const int qq = (y % p.r) * p.r + (x % p.r);
        return p.a + ((size_t)(b * (p.H / p.r) + y / p.r) * (p.W / p.r) + x / p.r) * p.ca +
               qq * p.c0 + c;
      }
      return p.b + ((size_t)(b * p.H + y) * p.W + x) * p.cb + (c - p.c0);
  }
}

// 8 consecutive channels [c, c+8) of the conv input at pixel (b, y, x) through
// the view (zero outside the image).
__device__ __forceinline__ bf16x8 view_chunk(const ConvArgs& p, int b, int y, int x, int c) {
  const uint16_t* ptr = view_ptr(p, b, y, x, c);
  return ptr ? ld8(ptr) : zero8();
}

__device__ __forceinline__ bf16x8 load_chunk(const ConvArgs& p, int b, int y, int x, int tap,
                                             int c) {
  if (tap >= p.taps) return zero8();
  if (p.taps == 9) {
    y += tap / 3 - 1;
    x += tap % 3 - 1;
  }
  return view_chunk(p, b, y, x, c);
}

// Accumulates the 32 x (16 NT) output tile of one wave over the whole K.
template <int NT>
__device__ __forceinline__ void conv_mainloop(const ConvArgs& p, int M, int m0, int n0, int lane,
                                              f32x4 (&acc)[2][NT]) {
  const int kq = lane >> 4, li = lane & 15;
  int pb[2], py[2], px[2];
  bool pv[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int m = m0 + r * 16 + li;
    pv[r] = m < M;
    const int mm = pv[r] ? m : 0;
    px[r] = mm % p.W;
    const int t = mm / p.W;
    py[r] = t % p.H;
    pb[r] = t / p.H;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int cpt = p.cin_p >> 3;  // 8-channel chunks per tap
  const uint16_t* wrow = p.w + (size_t)(n0 + li) * p.kp + kq * 8;
  // Operands of K step ks; the next step's loads are issued before this step's
  // MFMAs so that their latency overlaps the matrix work.
  auto load_step = [&](int ks, bf16x8 (&A)[2], bf16x8 (&Bv)[NT]) {
    const int q = (ks >> 3) + kq;
    const int tap = q / cpt;
    const int c = (q - tap * cpt) << 3;
#pragma unroll
    for (int r = 0; r < 2; ++r) A[r] = pv[r] ? load_chunk(p, pb[r], py[r], px[r], tap, c) : zero8();
#pragma unroll
    for (int j = 0; j < NT; ++j) Bv[j] = ld8(wrow + (size_t)j * 16 * p.kp + ks);
  };
  bf16x8 A[2], Bv[NT];
  load_step(0, A, Bv);
  for (int ks = 0; ks < p.kp; ks += 32) {
    bf16x8 An[2], Bn[NT];
    if (ks + 32 < p.kp) load_step(ks + 32, An, Bn);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
        acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], Bv[j], acc[r][j], 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 2; ++r) A[r] = An[r];
#pragma unroll
    for (int j = 0; j < NT; ++j) Bv[j] = Bn[j];
  }
}

// Epilogue of a wave's 32 x (16 NT) tile: bias, ReLU, residuals, FP32 and/or
// BF16 stores.  m[r][v] is the output pixel of accumulator row v of row tile r
// (-1: outside the image).  Every load (bias, residuals) is issued before the
// first store: the output pointers may alias nothing, but the compiler cannot
// know that, and interleaving would serialise one memory latency per element.
// The epilogue's first inputs (bias and the first residual), which a kernel
// may load before its main loop so that their latency overlaps the MFMAs.
template <int NT>
struct EpiIn {
  float bias[NT];
  float res[2][NT][4];
};

template <int NT>
__device__ __forceinline__ void epi_load(const ConvArgs& p, const int64_t (&m)[2][4], int n0,
                                         int li, EpiIn<NT>& in) {
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int n = n0 + j * 16 + li;
    in.bias[j] = n < p.cout ? p.bias[n] : 0.0f;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = n0 + j * 16 + li;
        in.res[r][j][v] = (p.res && m[r][v] >= 0 && n < p.cout)
                              ? p.res[(size_t)m[r][v] * p.cout + n] : 0.0f;
      }
}

template <int NT>
__device__ __forceinline__ void conv_epilogue(const ConvArgs& p, const f32x4 (&acc)[2][NT],
                                              const int64_t (&m)[2][4], int n0, int li,
                                              const EpiIn<NT>& in) {
  bool nv[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) nv[j] = n0 + j * 16 + li < p.cout;
  float y[2][NT][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float t = acc[r][j][v] + in.bias[j];
        y[r][j][v] = p.relu ? fmaxf(t, 0.0f) : t;
      }
  if (p.res) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) y[r][j][v] = in.res[r][j][v] + p.res_scale * y[r][j][v];
  }
  if (p.res2) {
    float rv[2][NT][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          rv[r][j][v] = (m[r][v] >= 0 && nv[j])
                            ? p.res2[(size_t)m[r][v] * p.cout + n0 + j * 16 + li] : 0.0f;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) y[r][j][v] += rv[r][j][v];
  }
  if (p.res3) {
    float rv[2][NT][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          rv[r][j][v] = (m[r][v] >= 0 && nv[j])
                            ? p.res3[(size_t)m[r][v] * p.cout + n0 + j * 16 + li] : 0.0f;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) y[r][j][v] += rv[r][j][v];
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (m[r][v] < 0 || !nv[j]) continue;
        const int n = n0 + j * 16 + li;
        if (p.out_f) p.out_f[(size_t)m[r][v] * p.out_f_stride + n] = y[r][j][v];
        if (p.out_h) p.out_h[(size_t)m[r][v] * p.out_h_stride + n] = f2bf(y[r][j][v]);
      }
}

// 3x3 convolution with its operands staged in LDS (gfx950 gives a workgroup up
// to 160 KB).  A block of 8 waves owns a 16 x 16 pixel tile of one image: the
// (16+2) x (16+2) x CINP input tile with its zero halo is gathered through the
// conv's input view (plain, or shuffle+concat), and the weights of one group
// of 16 NT output channels (9 CINP x 16 NT BF16) are loaded once per group;
// then every MFMA operand comes from LDS.  Wave w computes image rows 2w and
// 2w+1 of the tile (two 16-pixel row tiles) x 16 NT channels with
// v_mfma_f32_16x16x32_bf16; local K index k = tap CINP + c, so with CINP < 32
// one K step spans two taps.  Inputs wider than CINP (a multiple of it, CINP =
// 64: the dense blocks' 128..256-channel convs) are taken CINP channels at a
// time, tile and weights restaged per channel chunk, the accumulators kept.
// LDS layouts are chosen for conflict-free 16-byte accesses: tile pixels
// padded by 8 channels, weights chunk-major [k / 8][n][8] with one pad chunk
// per k row.
constexpr int C3_W = 16;  // tile width: one 16-pixel MFMA row tile

// Epilogue of a data-gradient conv with a plain backward (EPI_PLAIN of
// k_dgrad): y = scale acc (+ add1 + add2), zero where the ReLU mask is not
// positive, stored FP32 and/or BF16 (times out_h_scale).  Loads first, then
// stores, as in conv_epilogue.
__device__ __forceinline__ bool pos_bf(uint16_t h) { return h != 0 && !(h & 0x8000u); }

template <int NT>
__device__ __forceinline__ void dgrad_epilogue_plain(const BwdEpi& e, int cout,
                                                     const f32x4 (&acc)[2][NT],
                                                     const int64_t (&m)[2][4], int n0, int li) {
  float y[2][NT][4];
  bool keep[2][NT][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = n0 + j * 16 + li;
        keep[r][j][v] = m[r][v] >= 0 && n < cout;
        const size_t idx = keep[r][j][v] ? (size_t)m[r][v] * e.stride + n : 0;
        float t = acc[r][j][v] * e.scale;
        if (e.add1 && keep[r][j][v]) t += e.add1[idx];
        if (e.add2 && keep[r][j][v]) t += e.add2[idx];
        if (e.mask && keep[r][j][v] && !pos_bf(e.mask[idx])) t = 0.0f;
        y[r][j][v] = t;
      }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (!keep[r][j][v]) continue;
        const size_t idx = (size_t)m[r][v] * e.stride + n0 + j * 16 + li;
        if (e.out_f) e.out_f[idx] = y[r][j][v];
        if (e.out_h) e.out_h[idx] = f2bf(y[r][j][v] * e.out_h_scale);
      }
}

// LDS pitch of a tile pixel (BF16 channels): 16-byte reads of 8 consecutive
// lanes (pixels) at this stride hit distinct banks; a multiple of 32 channels
// needs 8 more (64: 72), other widths do not (80: 80, 16: 16, 8: 8).
template <int CINP>
constexpr int c3_pitch() {
  return CINP % 32 == 0 ? CINP + 8 : CINP;
}
// LDS bytes of a k_conv3_lds instance (input tile and weights).
template <int CINP, int NT, int TH>
constexpr int c3_lds_bytes() {
  constexpr int KP = (9 * CINP + 31) / 32 * 32;
  return 2 * ((TH + 2) * (C3_W + 2) * c3_pitch<CINP>() + (KP / 8) * (16 * NT + 1) * 8);
}
// Waves per SIMD the compiler must leave registers for (a block of TH / 2
// waves puts TH / 8 on each SIMD): two blocks per CU for the narrow convs (16
// output channels: the reconstruction convs) when the LDS allows it -- they fit
// in 128 VGPRs --, one block otherwise (the 64-channel instances need more
// registers than two blocks leave them, and spill when forced).
template <int CINP, int NT, int TH>
constexpr int c3_min_waves() {
  return (NT == 1 && c3_lds_bytes<CINP, NT, TH>() <= 80 * 1024 ? 2 : 1) *
         (TH / 8 > 0 ? TH / 8 : 1);
}

template <int CINP, int NT, int TH, bool DG = false>
__global__ __launch_bounds__(32 * TH, (c3_min_waves<CINP, NT, TH>())) void k_conv3_lds(
    ConvArgs p, int cout_p, int nsplit, BwdEpi be) {
  constexpr int THREADS = 32 * TH;  // TH / 2 waves, two tile rows each
  constexpr int TILE = (TH + 2) * (C3_W + 2);
  constexpr int PITCH = c3_pitch<CINP>();
  constexpr int KP = (9 * CINP + 31) / 32 * 32;
  constexpr int NG = 16 * NT;
  constexpr int WPITCH = NG + 1;  // 16-byte chunks per weight row (pad: conflict-free stores)
  constexpr int LDS_ALL = c3_lds_bytes<CINP, NT, TH>();
  __shared__ __attribute__((aligned(16))) uint16_t tile[TILE * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t wts[(KP / 8) * WPITCH * 8];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, li = lane & 15;
  const int x0 = blockIdx.x * C3_W, y0 = blockIdx.y * TH;
  const int b = blockIdx.z / nsplit, part = blockIdx.z - b * nsplit;
  const int nper = cout_p / nsplit;  // output channels of this block (a multiple of NG)
  const int nchunk = p.cin_p / CINP;
  // Loads are issued in batches (C3_BATCH_T tile chunks, C3_BATCH_W weight
  // chunks per thread) before their LDS stores, so that their latencies
  // overlap instead of adding up.
  constexpr int TCH = TILE * (CINP / 8), WCH = NG * (KP / 8);
  // A block whose LDS leaves room for no second block on its CU (more than
  // 80 KB) has 2 waves per SIMD, so registers are plentiful: 6 tile and 9
  // weight chunks in flight per thread; otherwise 3 and 3.
  constexpr int C3_BATCH_T = LDS_ALL > 80 * 1024 ? 6 : 3;
  constexpr int C3_BATCH_W = LDS_ALL > 80 * 1024 ? 9 : 3;
  for (int n0 = part * nper; n0 < (part + 1) * nper; n0 += NG) {
    f32x4 acc[2][NT];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ch = 0; ch < nchunk; ++ch) {
      const int cbase = ch * CINP;
      const bool first = n0 == part * nper && ch == 0;
      if (!first) __syncthreads();  // the LDS operands are no longer read
      if (nchunk > 1 || first) {
        auto tile_load = [&](int i) -> bf16x8 {
          const int px = i / (CINP / 8), c = (i - px * (CINP / 8)) * 8;
          const int ty = px / (C3_W + 2), tx = px - ty * (C3_W + 2);
          return i < TCH ? view_chunk(p, b, y0 - 1 + ty, x0 - 1 + tx, cbase + c) : zero8();
        };
        auto tile_store = [&](int i, bf16x8 v) {
          const int px = i / (CINP / 8), c = (i - px * (CINP / 8)) * 8;
          if (i < TCH) *reinterpret_cast<bf16x8*>(tile + px * PITCH + c) = v;
        };
        for (int i = tid; i < TCH; i += C3_BATCH_T * THREADS) {
          bf16x8 v[C3_BATCH_T];
#pragma unroll
          for (int u = 0; u < C3_BATCH_T; ++u) v[u] = tile_load(i + u * THREADS);
#pragma unroll
          for (int u = 0; u < C3_BATCH_T; ++u) tile_store(i + u * THREADS, v[u]);
        }
      }
      // local k = tap CINP + c holds packed column tap cin_p + cbase + c
      auto w_load = [&](int i) -> uint4 {
        const int n = i / (KP / 8), kc = i - n * (KP / 8);
        const int k = kc * 8, tap = k / CINP;
        const int kg = tap * p.cin_p + cbase + (k - tap * CINP);
        return i < WCH ? *reinterpret_cast<const uint4*>(p.w + (size_t)(n0 + n) * p.kp + kg)
                       : make_uint4(0u, 0u, 0u, 0u);
      };
      auto w_store = [&](int i, uint4 v) {
        const int n = i / (KP / 8), kc = i - n * (KP / 8);
        if (i < WCH) *reinterpret_cast<uint4*>(wts + (kc * WPITCH + n) * 8) = v;
      };
      for (int i = tid; i < WCH; i += C3_BATCH_W * THREADS) {
        uint4 v[C3_BATCH_W];
#pragma unroll
        for (int u = 0; u < C3_BATCH_W; ++u) v[u] = w_load(i + u * THREADS);
#pragma unroll
        for (int u = 0; u < C3_BATCH_W; ++u) w_store(i + u * THREADS, v[u]);
      }
      __syncthreads();
      for (int ks = 0; ks < KP; ks += 32) {
        const int k = ks + kq * 8;
        const int tap = k / CINP, c = k - tap * CINP;
        const int dy = tap / 3, dx = tap - dy * 3;
        bf16x8 A[2], Bv[NT];
#pragma unroll
        for (int r = 0; r < 2; ++r)
          A[r] = tap < 9 ? ld8(tile + ((2 * wave + r + dy) * (C3_W + 2) + li + dx) * PITCH + c)
                         : zero8();
#pragma unroll
        for (int j = 0; j < NT; ++j)
          Bv[j] = ld8(wts + (((ks >> 3) + kq) * WPITCH + j * 16 + li) * 8);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int j = 0; j < NT; ++j)
            acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], Bv[j], acc[r][j], 0, 0, 0);
      }
    }
    int64_t m[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int y = y0 + 2 * wave + r, x = x0 + kq * 4 + v;
        m[r][v] = (y < p.H && x < p.W) ? ((int64_t)b * p.H + y) * p.W + x : -1;
      }
    if (DG) {
      dgrad_epilogue_plain<NT>(be, p.cout, acc, m, n0, li);
    } else {
      EpiIn<NT> in;
      epi_load<NT>(p, m, n0, li, in);
      conv_epilogue<NT>(p, acc, m, n0, li, in);
    }
  }
}

// One residual block of the trunk in one launch: for a 16 x 16 output tile,
// y = res + res_scale convB(ReLU(convA(x))) (+ res2), convA and convB 3x3 convs
// of 64 channels.  The block stages x with a halo of 2, computes convA on the
// 18 x 18 pixels convB needs (halo recompute: 21 M tiles of 16 pixels instead
// of 16), keeps ReLU(convA) as BF16 in LDS -- zero outside the image, which is
// convB's zero padding -- and runs convB on it; convB's weights are loaded into
// registers during convA.  The intermediate is rounded to BF16 as the two-conv
// path stores it and every output element sums its K in the same order, so the
// result is bitwise that of convA then convB as two k_conv3_lds launches, less
// one launch and the intermediate's round trip through memory.
constexpr int RB_T = 16;          // output tile
constexpr int RB_IN = RB_T + 4;   // input tile rows / columns (halo of both convs)
constexpr int RB_MID = RB_T + 2;  // convA outputs = convB's input tile
constexpr int RB_C = 64;          // channels in and out of both convs
constexpr int RB_PITCH = RB_C + 8;
constexpr int RB_KP = 9 * RB_C;
constexpr int RB_WPITCH = RB_C + 1;  // 16-byte chunks per weight row
constexpr int RB_MIDT = (RB_MID * RB_MID + 15) / 16;  // convA's M tiles (21)
constexpr int RB_THREADS = 512;                      // 8 waves
constexpr int RB_MQ = (RB_MIDT + 7) / 8;             // convA M tiles per wave (3)

__global__ __launch_bounds__(RB_THREADS) void k_res_block(ConvArgs pa, ConvArgs pb) {
  __shared__ __attribute__((aligned(16))) uint16_t tile[RB_IN * RB_IN * RB_PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t wts[(RB_KP / 8) * RB_WPITCH * 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, li = lane & 15;
  const int x0 = blockIdx.x * RB_T, y0 = blockIdx.y * RB_T, b = blockIdx.z;
  constexpr int TCH = RB_IN * RB_IN * (RB_C / 8), WCH = RB_C * (RB_KP / 8);
  constexpr int WPT = WCH / RB_THREADS;  // weight chunks per thread (9)
  static_assert(WCH % RB_THREADS == 0, "weights split evenly over the threads");
  // input tile, 4 chunks in flight per thread
  for (int i = tid; i < TCH; i += 4 * RB_THREADS) {
    bf16x8 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ii = i + u * RB_THREADS, px = ii >> 3, c = (ii & 7) * 8;
      const int ty = px / RB_IN, tx = px - ty * RB_IN;
      v[u] = ii < TCH ? view_chunk(pa, b, y0 - 2 + ty, x0 - 2 + tx, c) : zero8();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ii = i + u * RB_THREADS;
      if (ii < TCH) *reinterpret_cast<bf16x8*>(tile + (ii >> 3) * RB_PITCH + (ii & 7) * 8) = v[u];
    }
  }
  // weights of chunk i: row n = i / (KP / 8), 16-byte chunk kc; LDS [kc][n][8]
  auto w_load = [&](const ConvArgs& p, int i) -> uint4 {
    const int n = i / (RB_KP / 8), kc = i - n * (RB_KP / 8);
    return *reinterpret_cast<const uint4*>(p.w + (size_t)n * p.kp + kc * 8);
  };
  auto w_store = [&](int i, uint4 v) {
    const int n = i / (RB_KP / 8), kc = i - n * (RB_KP / 8);
    *reinterpret_cast<uint4*>(wts + (kc * RB_WPITCH + n) * 8) = v;
  };
  {
    uint4 v[WPT];
#pragma unroll
    for (int u = 0; u < WPT; ++u) v[u] = w_load(pa, tid + u * RB_THREADS);
#pragma unroll
    for (int u = 0; u < WPT; ++u) w_store(tid + u * RB_THREADS, v[u]);
  }
  __syncthreads();
  // convB's weights, in flight while convA runs
  uint4 wb[WPT];
#pragma unroll
  for (int u = 0; u < WPT; ++u) wb[u] = w_load(pb, tid + u * RB_THREADS);
  // convA: wave w takes M tiles w, w + 8, w + 16 of the 18 x 18 intermediate
  // pixels in row-major order; lane li holds pixel 16 t + li of the A operand
  f32x4 acc[RB_MQ][4];
  int pofs[RB_MQ];
#pragma unroll
  for (int q = 0; q < RB_MQ; ++q) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[q][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int pix = 16 * (wave + 8 * q) + li;
    const int iy = pix / RB_MID, ix = pix - iy * RB_MID;
    pofs[q] = pix < RB_MID * RB_MID ? (iy * RB_IN + ix) * RB_PITCH : -1;
  }
  for (int ks = 0; ks < RB_KP; ks += 32) {
    const int k = ks + kq * 8;
    const int tap = k / RB_C, c = k - tap * RB_C;
    const int dy = tap / 3, dx = tap - dy * 3;
    const int tofs = (dy * RB_IN + dx) * RB_PITCH + c;
    bf16x8 Bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) Bv[j] = ld8(wts + (((ks >> 3) + kq) * RB_WPITCH + j * 16 + li) * 8);
#pragma unroll
    for (int q = 0; q < RB_MQ; ++q) {
      if (wave + 8 * q >= RB_MIDT) continue;  // wave-uniform
      const bf16x8 A = pofs[q] >= 0 ? ld8(tile + pofs[q] + tofs) : zero8();
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv[j], acc[q][j], 0, 0, 0);
    }
  }
  // ReLU(convA + bias) as BF16, zero outside the image and past the 18 x 18
  uint16_t hv[RB_MQ][4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float bias = pa.bias[j * 16 + li];
#pragma unroll
    for (int q = 0; q < RB_MQ; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pix = 16 * (wave + 8 * q) + kq * 4 + v;
        const int iy = pix / RB_MID, ix = pix - iy * RB_MID;
        const int y = y0 - 1 + iy, x = x0 - 1 + ix;
        const bool in = pix < RB_MID * RB_MID && y >= 0 && y < pa.H && x >= 0 && x < pa.W;
        hv[q][j][v] = in ? f2bf(fmaxf(acc[q][j][v] + bias, 0.0f)) : (uint16_t)0;
      }
  }
  __syncthreads();  // convA's operands are no longer read
#pragma unroll
  for (int q = 0; q < RB_MQ; ++q) {
    if (wave + 8 * q >= RB_MIDT) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int pix = 16 * (wave + 8 * q) + kq * 4 + v;
      if (pix >= RB_MID * RB_MID) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) tile[pix * RB_PITCH + j * 16 + li] = hv[q][j][v];
    }
  }
#pragma unroll
  for (int u = 0; u < WPT; ++u) w_store(tid + u * RB_THREADS, wb[u]);
  __syncthreads();
  // convB on the 16 x 16 tile: wave w computes rows 2w and 2w + 1
  f32x4 acc2[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc2[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < RB_KP; ks += 32) {
    const int k = ks + kq * 8;
    const int tap = k / RB_C, c = k - tap * RB_C;
    const int dy = tap / 3, dx = tap - dy * 3;
    bf16x8 A[2], Bv[4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
      A[r] = ld8(tile + ((2 * wave + r + dy) * RB_MID + li + dx) * RB_PITCH + c);
#pragma unroll
    for (int j = 0; j < 4; ++j) Bv[j] = ld8(wts + (((ks >> 3) + kq) * RB_WPITCH + j * 16 + li) * 8);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc2[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], Bv[j], acc2[r][j], 0, 0, 0);
  }
  int64_t m[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int y = y0 + 2 * wave + r, x = x0 + kq * 4 + v;
      m[r][v] = (y < pb.H && x < pb.W) ? ((int64_t)b * pb.H + y) * pb.W + x : -1;
    }
  EpiIn<4> in;
  epi_load<4>(pb, m, 0, li, in);
  conv_epilogue<4>(pb, acc2, m, 0, li, in);
}

// Runs the conv on k_conv3_lds<CINP, NT, TH> if its shape fits: cin_p == CINP,
// or (CINP = 64) a multiple of it taken in chunks; packed K = 9 cin_p rounded up
// to 32; cout_p a multiple of nsplit channel groups of 16 NT.  The output
// channels are split over nsplit blocks per tile.
template <int CINP, int NT, int TH, bool DG = false>
bool try_conv3_lds(const ConvArgs& a, int cout_p, int nsplit, hipStream_t st,
                   const BwdEpi* be = nullptr) {
  const bool chunked = CINP == 64 && a.cin_p > CINP && a.cin_p % CINP == 0;
  if ((a.cin_p != CINP && !chunked) || a.kp != (9 * a.cin_p + 31) / 32 * 32 ||
      cout_p % (16 * NT * nsplit))
    return false;
  BwdEpi e;
  if (be) e = *be;
  else std::memset(&e, 0, sizeof e);
  k_conv3_lds<CINP, NT, TH, DG><<<dim3((a.W + C3_W - 1) / C3_W, (a.H + TH - 1) / TH,
                                       a.B * nsplit),
                                  32 * TH, 0, st>>>(a, cout_p, nsplit, e);
  return true;
}

template <int NT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs p) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int M = p.B * p.H * p.W;
  const int m0 = (blockIdx.x * 4 + wave) * 32;
  if (m0 >= M) return;
  const int n0 = blockIdx.y * (NT * 16);
  f32x4 acc[2][NT];
  conv_mainloop<NT>(p, M, m0, n0, lane, acc);
  const int kq = lane >> 4, li = lane & 15;
  int64_t m[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int mm = m0 + r * 16 + kq * 4 + v;
      m[r][v] = mm < M ? mm : -1;
    }
  EpiIn<NT> in;
  epi_load<NT>(p, m, n0, li, in);
  conv_epilogue<NT>(p, acc, m, n0, li, in);
}

// Data gradient of a conv: the same implicit GEMM over dY with the packed
// transposed, flipped weights; the epilogue applies the backward of what
// surrounds the conv (ReLU masks, residual sums, the (un)shuffle views).
template <int NT>
__global__ __launch_bounds__(256) void k_dgrad(ConvArgs p, BwdEpi e) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int M = p.B * p.H * p.W;
  const int m0 = (blockIdx.x * 4 + wave) * 32;
  if (m0 >= M) return;
  const int n0 = blockIdx.y * (NT * 16);
  f32x4 acc[2][NT];
  conv_mainloop<NT>(p, M, m0, n0, lane, acc);
  const int kq = lane >> 4, li = lane & 15;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int n = n0 + j * 16 + li;
      if (n >= p.cout) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + r * 16 + kq * 4 + v;
        if (m >= M) continue;
        float y = acc[r][j][v] * e.scale;
        if (e.mode == EPI_PLAIN) {
          const size_t idx = (size_t)m * e.stride + n;
          if (e.add1) y += e.add1[idx];
          if (e.add2) y += e.add2[idx];
          if (e.mask && !pos_bf(e.mask[idx])) y = 0.0f;
          if (e.out_f) e.out_f[idx] = y;
          if (e.out_h) e.out_h[idx] = f2bf(y * e.out_h_scale);
        } else if (e.mode == EPI_REC_SPLIT) {  // this conv at HR; [shuffle(U) | h0]
          const int x = m % p.W, t = m / p.W, yy = t % p.H, b = t / p.H;
          if (n < e.c_split) {
            const int hh = p.H / e.r, ww = p.W / e.r;
            const size_t idx = ((size_t)(b * hh + yy / e.r) * ww + x / e.r) * e.stride2 +
                               ((yy % e.r) * e.r + (x % e.r)) * e.c_split + n;
            if (!pos_bf(e.mask[idx])) y = 0.0f;
            e.out_h[idx] = f2bf(y);
          } else {
            e.out_f[(size_t)m * e.stride + (n - e.c_split)] = y;
          }
        } else if (e.mode == EPI_FUSE_SPLIT) {  // this conv at LR; [fl | unshuffle(h0)]
          if (n < e.c_split) {
            const size_t idx = (size_t)m * e.c_split + n;
            if (!pos_bf(e.mask[idx])) y = 0.0f;
            e.out_h[idx] = f2bf(y);
          } else {
            const int X = m % p.W, t = m / p.W, Y = t % p.H, b = t / p.H;
            const int cc = n - e.c_split, q = cc / e.stride, ch = cc - q * e.stride;
            int I, J;
            unshuffle_slot(q, e.r, e.dsf, I, J);
            const int hy = Y * e.r + I, hx = X * e.r + J;
            const size_t hidx = ((size_t)(b * p.H * e.r + hy) * (p.W * e.r) + hx) * e.stride + ch;
            float v2 = e.add1 ? y + e.add1[hidx] : y;
            if (!pos_bf(e.mask2[hidx])) v2 = 0.0f;
            e.out_h2[hidx] = f2bf(v2);
          }
        } else {  // EPI_DENSE: input slices 0 .. k-1 of a residual dense block
          const int sl = n >> 6, ch = n & 63;
          const size_t gi = (size_t)m * RDG_DENSE + n, i64 = (size_t)m * NET_FEAT + ch;
          if (e.k == 1) {  // x_0 complete: the gradient of the block input
            y += e.ga[gi];
            if (e.add1) y += e.add1[i64];
            if (e.add2) y += e.add2[i64];
            if (e.mask0 && !pos_bf(e.dense[gi])) y = 0.0f;
            if (e.out_f) e.out_f[i64] = y;
            e.out_h[i64] = f2bf(y);
          } else if (sl == e.k - 1) {  // x_{k-1} complete: through its ReLU
            if (!e.fusing) y += e.ga[gi];
            if (!pos_bf(e.dense[gi])) y = 0.0f;
            e.dy_next[i64] = f2bf(y);
          } else if (e.fusing) {
            if (sl == 0) y += e.ds[i64];
            e.ga[gi] = y;
          } else {
            e.ga[gi] += y;
          }
        }
      }
    }
  }
}

// Network inputs: HRLS -> 16 BF16 channels (log1p of clipped RGB, albedo,
// normal, log1p depth, 6 zeros); LRHS -> 8 channels (log1p RGB, 5 zeros).
__global__ __launch_bounds__(256) void k_prep(int64_t nhr, int64_t nlr,
                                              const float* __restrict__ hr,
                                              const float* __restrict__ aux,
                                              const float* __restrict__ lr,
                                              uint16_t* __restrict__ xh,
                                              uint16_t* __restrict__ xl) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nhr) {
    float v[16];
    for (int c = 0; c < 3; ++c) v[c] = log1pf(fminf(fmaxf(hr[3 * i + c], 0.0f), 100.0f));
    for (int c = 0; c < 6; ++c) v[3 + c] = aux[7 * i + c];
    v[9] = log1pf(fmaxf(aux[7 * i + 6], 0.0f));
    for (int c = 10; c < 16; ++c) v[c] = 0.0f;
    uint32_t w[8];
    for (int k = 0; k < 8; ++k) w[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
    uint4* o = reinterpret_cast<uint4*>(xh + 16 * i);
    o[0] = make_uint4(w[0], w[1], w[2], w[3]);
    o[1] = make_uint4(w[4], w[5], w[6], w[7]);
  } else if (i < nhr + nlr) {
    const int64_t j = i - nhr;
    float v[8];
    for (int c = 0; c < 3; ++c) v[c] = log1pf(fminf(fmaxf(lr[3 * j + c], 0.0f), 100.0f));
    for (int c = 3; c < 8; ++c) v[c] = 0.0f;
    uint32_t w[4];
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
    *reinterpret_cast<uint4*>(xl + 8 * j) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Network inputs with the HRLS render layers: HRLS -> 16 BF16 channels (log1p
// of clipped RGB, albedo, normal, log1p of the clipped diffuse and glossy
// layers, log1p of the per-sample variance averaged over RGB, clamped to
// [0, 1e4]); LRHS as in k_prep.
__global__ __launch_bounds__(256) void k_prep_layers(int64_t nhr, int64_t nlr,
                                                     const float* __restrict__ hr,
                                                     const float* __restrict__ aux,
                                                     const float* __restrict__ lay,
                                                     const float* __restrict__ sq, float inv_spp,
                                                     const float* __restrict__ lr,
                                                     uint16_t* __restrict__ xh,
                                                     uint16_t* __restrict__ xl) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nhr) {
    float v[16];
    float var = 0.0f;
    for (int c = 0; c < 3; ++c) {
      const float m = hr[3 * i + c];
      v[c] = log1pf(fminf(fmaxf(m, 0.0f), 100.0f));
      var += sq[3 * i + c] * inv_spp - m * m;
    }
    for (int c = 0; c < 6; ++c) v[3 + c] = aux[7 * i + c];
    for (int c = 0; c < 6; ++c) v[9 + c] = log1pf(fminf(fmaxf(lay[9 * i + 3 + c], 0.0f), 100.0f));
    v[15] = log1pf(fminf(fmaxf(var * (1.0f / 3.0f), 0.0f), 1.0e4f));
    uint32_t w[8];
    for (int k = 0; k < 8; ++k) w[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
    uint4* o = reinterpret_cast<uint4*>(xh + 16 * i);
    o[0] = make_uint4(w[0], w[1], w[2], w[3]);
    o[1] = make_uint4(w[4], w[5], w[6], w[7]);
  } else if (i < nhr + nlr) {
    const int64_t j = i - nhr;
    float v[8];
    for (int c = 0; c < 3; ++c) v[c] = log1pf(fminf(fmaxf(lr[3 * j + c], 0.0f), 100.0f));
    for (int c = 3; c < 8; ++c) v[c] = 0.0f;
    uint32_t w[4];
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
    *reinterpret_cast<uint4*>(xl + 8 * j) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// BF16 weight packing of every layer in one launch (master layout
// [cout][cin][k][k]).  Element i belongs to the last job whose begin is <= i.
// t = 0: wp[n][tap cin_p + c] = W[n][c][tap], the forward convs' B operand.
// t = 1: wt[c][tap' cinp_t + n] = W[n][c][taps - 1 - tap'], the data-gradient
// conv (flipped taps, input and output channels swapped).  Padding is zero.
__global__ __launch_bounds__(256) void k_pack_all(const float* __restrict__ wm,
                                                  const PackJob* __restrict__ jobs, int njobs,
                                                  int64_t total, uint16_t* __restrict__ packed,
                                                  uint16_t* __restrict__ packed_t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].begin <= i) lo = mid;
    else hi = mid - 1;
  }
  const PackJob& J = jobs[lo];
  const int64_t e = i - J.begin;
  const int row = (int)(e / J.kp), k = (int)(e % J.kp);
  const int tap = k / J.cinp, col = k % J.cinp;
  const int taps = J.ksz * J.ksz;
  const float* w = wm + J.w_off;
  float v = 0.0f;
  if (J.t == 0) {  // row = output channel n, col = input channel c
    if (row < J.cout && col < J.cin && tap < taps)
      v = w[((size_t)(row * J.cin + col) * taps) + tap];
    packed[J.out_off + e] = f2bf(v);
  } else {  // row = input channel c, col = output channel n, flipped tap
    if (row < J.cin && col < J.cout && tap < taps)
      v = w[((size_t)(col * J.cin + row) * taps) + (taps - 1 - tap)];
    packed_t[J.out_off + e] = f2bf(v);
  }
}

// He-uniform initialisation (fan-in), Philox4x32-10 with tag 2; biases 0.
__global__ __launch_bounds__(256) void k_init(float* __restrict__ dst, int64_t nw, int64_t nb,
                                              int64_t first, float bound, uint32_t k0,
                                              uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nw) {
    const int64_t g = first + i;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)(g >> 32), 0u, 2u), k0, k1);
    dst[i] = (2.0f * unit24(r.x) - 1.0f) * bound;
  } else if (i < nw + nb) {
    dst[i] = 0.0f;
  }
}

// Weight gradient on the matrix cores, split over pixels: part[s][n][col] = sum
// over the pixels of split s of dY[p][n] X[p + off(tap)][c], col = tap cin_p + c
// (the packed K layout).  The pixel is the MFMA's K index: lane (i, kq) of a
// wave reads, for the pixels p0 + 8 kq + e (e < 8) of each 32-pixel step, RN
// channels of dY and QX columns of X with one load each, and re-packs the
// 16-bit halves into operands: dY operand c maps row i to channel n0 + RN i + c
// (RN = 1: channel n0 + i), X operand d maps column i to col0 + QX i + d.  No LDS
// staging and no barrier in the loop; the next step's loads are issued before
// this step's MFMAs.  The 4 waves of a workgroup take consecutive quarters of
// the split's pixels and their tiles are summed in LDS in wave order
// (deterministic).  The first column block also sums dY, the bias gradient.
// FAST: plain view and W % 8 == 0, so a lane's 8 pixels share one image row.
template <int W>
struct Dw {
  uint32_t v[W];
};

template <int W>
__device__ __forceinline__ Dw<W> ldw(const uint16_t* p) {
  Dw<W> r;
  if constexpr (W == 1) {
    r.v[0] = *reinterpret_cast<const uint32_t*>(p);
  } else if constexpr (W == 2) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    r.v[0] = u.x;
    r.v[1] = u.y;
  } else {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    r.v[0] = u.x;
    r.v[1] = u.y;
    r.v[2] = u.z;
    r.v[3] = u.w;
  }
  return r;
}

template <int W>
__device__ __forceinline__ Dw<W> zdw() {
  Dw<W> r;
#pragma unroll
  for (int k = 0; k < W; ++k) r.v[k] = 0u;
  return r;
}

// The 16-bit half at bit `sh` (0 or 16) of word u of pixels 2k and 2k+1, packed
// into one operand word (pixel 2k low).
__device__ __forceinline__ uint32_t pair16(uint32_t lo, uint32_t hi, int sh) {
  return ((lo >> sh) & 0xffffu) | ((hi >> sh) << 16);
}

template <int RN, int QX, bool FAST>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  constexpr int NN = 16 * RN, NC = 16 * QX;
  constexpr int YW = RN == 1 ? 1 : RN / 2, XW = QX / 2;  // dwords per pixel
  __shared__ __attribute__((aligned(16))) float red[4][NN * NC];
  __shared__ float bred[4][NN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int col0 = blockIdx.x * NC, n0 = blockIdx.y * NN;
  const ConvArgs& x = a.x;
  const int quarter = a.chunk >> 2;
  const int pw0 = blockIdx.z * a.chunk + wave * quarter;
  const int pw1 = min(a.npix, pw0 + quarter);
  // this lane's X columns: QX channels cx.. of tap `tap` (one tap: cin_p % 8 == 0)
  const int colx = col0 + QX * i;
  const int tapx = colx / x.cin_p, cx = colx - tapx * x.cin_p;
  const bool xon = colx < x.kp && tapx < x.taps;
  const int ty = x.taps == 9 ? tapx / 3 - 1 : 0, tx = x.taps == 9 ? tapx % 3 - 1 : 0;
  // this lane's dY channels (RN = 1: the word holding channel n0 + i)
  const int ny = RN == 1 ? ((n0 + i) & ~1) : n0 + RN * i;
  const bool yon = (RN == 1 ? n0 + i : ny) < a.dy_stride;
  const int ysh = RN == 1 ? 16 * ((n0 + i) & 1) : 0;
  const bool bias_blk = blockIdx.x == 0 && a.bpart;

  auto load_step = [&](int pk, Dw<YW>(&yd)[8], Dw<XW>(&xd)[8]) {
    const int pp0 = pk + 8 * kq;
    const uint16_t* yp = a.dy + (int64_t)pp0 * a.dy_stride + ny;
    if constexpr (FAST) {
      const bool gv = pp0 < pw1;  // W % 8 == 0: the 8 pixels are valid together
      const int x0 = pp0 % x.W, y0 = (pp0 / x.W) % x.H;
      const bool rowv = gv && xon && (unsigned)(y0 + ty) < (unsigned)x.H;
      const uint16_t* xp = x.a + ((int64_t)pp0 + ty * x.W + tx) * x.ca + cx;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool xv = rowv && (unsigned)(x0 + e + tx) < (unsigned)x.W;
        xd[e] = xv ? ldw<XW>(xp + (int64_t)e * x.ca) : zdw<XW>();
        yd[e] = (gv && yon) ? ldw<YW>(yp + (int64_t)e * a.dy_stride) : zdw<YW>();
      }
    } else {
      int px = pp0 % x.W;
      const int t = pp0 / x.W;
      int py = t % x.H, pb = t / x.H;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool v = pp0 + e < pw1;
        const uint16_t* q = (v && xon) ? view_ptr(x, pb, py + ty, px + tx, cx) : nullptr;
        xd[e] = q ? ldw<XW>(q) : zdw<XW>();
        yd[e] = (v && yon) ? ldw<YW>(yp + (int64_t)e * a.dy_stride) : zdw<YW>();
        ++px;
        const bool wrap = px == x.W;
        px = wrap ? 0 : px;
        py += wrap;
        const bool wrap2 = py == x.H;
        py = wrap2 ? 0 : py;
        pb += wrap2;
      }
    }
  };

  f32x4 acc[RN][QX];
#pragma unroll
  for (int c = 0; c < RN; ++c)
#pragma unroll
    for (int d = 0; d < QX; ++d) acc[c][d] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bs[RN];
#pragma unroll
  for (int c = 0; c < RN; ++c) bs[c] = 0.0f;

  Dw<YW> yd[8];
  Dw<XW> xd[8];
  if (pw0 < pw1) load_step(pw0, yd, xd);
  for (int pk = pw0; pk < pw1; pk += 32) {
    Dw<YW> yn[8];
    Dw<XW> xn[8];
    if (pk + 32 < pw1) load_step(pk + 32, yn, xn);
    bf16x8 A[RN], Bv[QX];
#pragma unroll
    for (int c = 0; c < RN; ++c) {
      const int u = RN == 1 ? 0 : c >> 1, sh = RN == 1 ? ysh : 16 * (c & 1);
      uint4 w;
      w.x = pair16(yd[0].v[u], yd[1].v[u], sh);
      w.y = pair16(yd[2].v[u], yd[3].v[u], sh);
      w.z = pair16(yd[4].v[u], yd[5].v[u], sh);
      w.w = pair16(yd[6].v[u], yd[7].v[u], sh);
      A[c] = __builtin_bit_cast(bf16x8, w);
      if (bias_blk) {
#pragma unroll
        for (int e = 0; e < 8; ++e) bs[c] += __uint_as_float(((yd[e].v[u] >> sh) & 0xffffu) << 16);
      }
    }
#pragma unroll
    for (int d = 0; d < QX; ++d) {
      const int u = d >> 1, sh = 16 * (d & 1);
      uint4 w;
      w.x = pair16(xd[0].v[u], xd[1].v[u], sh);
      w.y = pair16(xd[2].v[u], xd[3].v[u], sh);
      w.z = pair16(xd[4].v[u], xd[5].v[u], sh);
      w.w = pair16(xd[6].v[u], xd[7].v[u], sh);
      Bv[d] = __builtin_bit_cast(bf16x8, w);
    }
#pragma unroll
    for (int c = 0; c < RN; ++c)
#pragma unroll
      for (int d = 0; d < QX; ++d)
        acc[c][d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[c], Bv[d], acc[c][d], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      yd[e] = yn[e];
      xd[e] = xn[e];
    }
  }
  // accumulator (c, d) of lane (j, g): rows 4g + v (channel n0 + RN row + c),
  // column j (col0 + QX j + d)
  {
    const int j = lane & 15, g = lane >> 4;
    float* r = red[wave];
#pragma unroll
    for (int c = 0; c < RN; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float* row = r + (RN * (4 * g + v) + c) * NC + QX * j;
#pragma unroll
        for (int d4 = 0; d4 < QX; d4 += 4)
          *reinterpret_cast<float4*>(row + d4) =
              make_float4(acc[c][d4][v], acc[c][d4 + 1][v], acc[c][d4 + 2][v], acc[c][d4 + 3][v]);
      }
  }
  if (bias_blk) {  // over kq (lanes 16 apart), then per wave into LDS
#pragma unroll
    for (int c = 0; c < RN; ++c) {
      bs[c] += __shfl_xor(bs[c], 16);
      bs[c] += __shfl_xor(bs[c], 32);
    }
    if (kq == 0) {
#pragma unroll
      for (int c = 0; c < RN; ++c) bred[wave][RN == 1 ? i : RN * i + c] = bs[c];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  float* out = a.part + ((size_t)blockIdx.z * a.cout_p + n0) * x.kp + col0;
  for (int f = t; f < NN * NC / 4; f += 256) {
    const int nl = (4 * f) / NC, cl = (4 * f) % NC;
    if (col0 + cl >= x.kp) continue;
    const float4 r0 = reinterpret_cast<const float4*>(red[0])[f];
    const float4 r1 = reinterpret_cast<const float4*>(red[1])[f];
    const float4 r2 = reinterpret_cast<const float4*>(red[2])[f];
    const float4 r3 = reinterpret_cast<const float4*>(red[3])[f];
    *reinterpret_cast<float4*>(out + (size_t)nl * x.kp + cl) =
        make_float4(((r0.x + r1.x) + r2.x) + r3.x, ((r0.y + r1.y) + r2.y) + r3.y,
                    ((r0.z + r1.z) + r2.z) + r3.z, ((r0.w + r1.w) + r2.w) + r3.w);
  }
  if (bias_blk && t < NN && n0 + t < a.cout)
    a.bpart[(size_t)blockIdx.z * a.cout + n0 + t] =
        ((bred[0][t] + bred[1][t]) + bred[2][t]) + bred[3][t];
}

// Sum of v[sp * stride] over the splits: eight independent partial sums
// (split sp into sum sp % 8), so that eight loads are in flight, then added in a
// fixed order.
__device__ __forceinline__ float sum_splits(const float* __restrict__ v, size_t stride,
                                            int splits) {
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int sp = 0;
  for (; sp + 8 <= splits; sp += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] += v[(size_t)(sp + k) * stride];
  }
  for (int k = 0; sp < splits; ++sp, ++k) s[k] += v[(size_t)sp * stride];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Sum the split partials in order and scatter into the master gradient layout
// [cout][cin][k][k] followed by the bias.  Threads walk the packed layout
// [n][tap cin_p + c], so that the split partials are read coalesced.
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ part,
                                                     const float* __restrict__ bpart, int splits,
                                                     int cout, int cin, int ksz, int cin_p, int kp,
                                                     int cout_p, float* __restrict__ g) {
  const int64_t np = (int64_t)cout * kp;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < np) {
    const int n = (int)(i / kp), col = (int)(i - (int64_t)n * kp);
    const int tap = col / cin_p, c = col - tap * cin_p;
    if (c >= cin || tap >= ksz * ksz) return;
    const int ky = tap / ksz, kx = tap - ky * ksz;
    g[((size_t)(n * cin + c) * ksz + ky) * ksz + kx] =
        sum_splits(part + i, (size_t)cout_p * kp, splits);
  } else if (i < np + cout) {
    const int n = (int)(i - np);
    g[(size_t)cout * cin * ksz * ksz + n] = sum_splits(bpart + n, (size_t)cout, splits);
  }
}

// Loss pieces (t clipped to [0, 100], d = y - t).  beta <= 0: L1, FP64 partial
// sums of |d| per block and the gradient sign(d) / N.  beta > 0: the robust loss
// of Sec. 4, partial sums of |d| / (beta + |d|) in FP64 and the gradient
// sign(d) beta / (beta + |d|)^2 / N.  sign(0) = 0; the gradient is stored as
// BF16 in an 8-channel padded tensor.
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ y,
                                            const float* __restrict__ tgt, int64_t npix,
                                            double inv_n, float beta, double* __restrict__ part,
                                            uint16_t* __restrict__ g8) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix;
       p += (int64_t)gridDim.x * 256) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (int c = 0; c < 3; ++c) {
      // targets are clipped to [0, 100] like the training data (fireflies, Sec. 3.2)
      const float d = y[3 * p + c] - fminf(fmaxf(tgt[3 * p + c], 0.0f), 100.0f);
      const double ad = fabs((double)d);
      const float gsgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
      float gv;
      if (beta > 0.0f) {
        s += ad / ((double)beta + ad);
        const float den = beta + fabsf(d);
        gv = gsgn * (beta / (den * den)) * (float)inv_n;
      } else {
        s += ad;
        gv = gsgn * (float)inv_n;
      }
      const uint32_t h = f2bf(gv);
      w[c >> 1] |= h << (16 * (c & 1));
    }
    *reinterpret_cast<uint4*>(g8 + 8 * p) = make_uint4(w[0], w[1], w[2], w[3]);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_l1_final(const double* __restrict__ part, int nparts,
                                                  double inv_n, double* __restrict__ loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) s += part[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] * inv_n;
}

// A caller-supplied output gradient (FP32 [P][3]) as BF16 in the 8-channel
// padded layout the backward pass reads.
__global__ __launch_bounds__(256) void k_grad_in(const float* __restrict__ gout, int64_t npix,
                                                 uint16_t* __restrict__ g8) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const uint32_t w0 = (uint32_t)f2bf(gout[3 * p]) | ((uint32_t)f2bf(gout[3 * p + 1]) << 16);
  const uint32_t w1 = (uint32_t)f2bf(gout[3 * p + 2]);
  *reinterpret_cast<uint4*>(g8 + 8 * p) = make_uint4(w0, w1, 0u, 0u);
}

// Plain SGD on the FP32 masters (the paper's optimiser): w -= lr g.
__global__ __launch_bounds__(256) void k_sgd(float* __restrict__ w, const float* __restrict__ g,
                                             int64_t n, float lr) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) w[i] -= lr * g[i];
}

// Adam (Kingma & Ba 2015, Algorithm 1) on the FP32 masters; c1 = 1 - b1^t,
// c2 = 1 - b2^t are the bias corrections of step t.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

namespace {
inline unsigned cdiv64(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
}  // namespace

namespace {
std::atomic<int64_t> g_conv_launches[MRS_NUM_CONV_KINDS];
inline void count_conv(int kind) { g_conv_launches[kind].fetch_add(1, std::memory_order_relaxed); }
}  // namespace

void launch_dgrad(const ConvArgs& a, const BwdEpi& e, int cout_p, hipStream_t st) {
  // 3x3 data gradients with a plain backward on the LDS conv (the same tile
  // plans as the forward convs)
  if (e.mode == EPI_PLAIN && a.taps == 9 && a.mode == VIEW_PLAIN && a.ca >= a.cin_p &&
      cout_p >= 64 && a.cin_p % 64 == 0) {
    const int64_t tiles = (int64_t)((a.W + 15) / 16) * ((a.H + 15) / 16) * a.B;
    if (tiles < conv_small_tiles() && try_conv3_lds<64, 2, 8, true>(a, cout_p, cout_p / 32, st, &e))
      return count_conv(8);
    if (try_conv3_lds<64, 4, 16, true>(a, cout_p, 1, st, &e)) return count_conv(9);
  }
  const int64_t M = (int64_t)a.B * a.H * a.W;
  const unsigned gx = cdiv64(M, 128);
  if (cout_p >= 64) {
    k_dgrad<4><<<dim3(gx, cout_p / 64), 256, 0, st>>>(a, e);
  } else {
    k_dgrad<1><<<dim3(gx, cout_p / 16), 256, 0, st>>>(a, e);
  }
}

// Weight-gradient tile per workgroup: 64 x 64 (RN 4, QX 4) for 64 or more
// output channels, else 16 x 128 (RN 1, QX 8).
namespace {
inline int wgrad_nc(int cout_p) { return cout_p >= 64 ? 64 : 128; }
inline int wgrad_nn(int cout_p) { return cout_p >= 64 ? 64 : 16; }
}  // namespace

int wgrad_splits(int64_t npix, int kp, int cout_p, int& chunk) {
  // about 1024 workgroups over the tiles, at most 128 splits, and at least 4
  // steps of 32 pixels per wave (512 pixels per workgroup)
  const int64_t tiles = (int64_t)cdiv64(kp, wgrad_nc(cout_p)) * (cout_p / wgrad_nn(cout_p));
  const int64_t s = std::max<int64_t>(1, std::min<int64_t>(128, (1024 + tiles - 1) / tiles));
  const int64_t per = std::max<int64_t>(512, (npix + s - 1) / s);
  chunk = (int)((per + 127) / 128 * 128);
  return (int)std::max<int64_t>(1, (npix + chunk - 1) / chunk);
}

void launch_wgrad(const WgradArgs& a, int splits, hipStream_t st) {
  const bool fast = a.x.mode == VIEW_PLAIN && a.x.W % 8 == 0;
  const dim3 grid(cdiv64(a.x.kp, wgrad_nc(a.cout_p)), a.cout_p / wgrad_nn(a.cout_p), splits);
  if (a.cout_p >= 64) {
    if (fast)
      k_wgrad<4, 4, true><<<grid, 256, 0, st>>>(a);
    else
      k_wgrad<4, 4, false><<<grid, 256, 0, st>>>(a);
  } else {
    if (fast)
      k_wgrad<1, 8, true><<<grid, 256, 0, st>>>(a);
    else
      k_wgrad<1, 8, false><<<grid, 256, 0, st>>>(a);
  }
}

void launch_grad_reduce(const float* part, const float* bpart, int splits, const NetLayer& L,
                        float* g, hipStream_t st) {
  const int64_t n = (int64_t)L.cout * L.kp + L.cout;
  k_grad_reduce<<<cdiv64(n, 256), 256, 0, st>>>(part, bpart, splits, L.cout, L.cin, L.k, L.cin_p,
                                                 L.kp, L.cout_p, g);
}

void launch_out_grad(const OutGrad& o, const float* y, int64_t npix, uint16_t* g8,
                     hipStream_t st) {
  if (o.tgt) {
    const double inv_n = 1.0 / (double)(3 * npix);
    k_l1<<<o.nparts, 256, 0, st>>>(y, o.tgt, npix, inv_n, o.beta, o.part, g8);
    k_l1_final<<<1, 256, 0, st>>>(o.part, o.nparts, inv_n, o.loss);
  } else {
    k_grad_in<<<cdiv64(npix, 256), 256, 0, st>>>(o.gout, npix, g8);
  }
}

void launch_sgd(float* w, const float* g, int64_t n, float lr, hipStream_t st) {
  k_sgd<<<cdiv64(n, 256), 256, 0, st>>>(w, g, n, lr);
}

void launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st) {
  k_adam<<<cdiv64(n, 256), 256, 0, st>>>(w, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

// Tile plan of a 3x3 conv on k_conv3_lds: 16 x 16 tiles of 8 waves with all
// output channels per block; when such tiles are fewer than
// mrs_tuning.conv_small_tiles (default 128: half of the 256 CUs), 16 x 8 tiles
// of 4 waves with the output channels split over blocks of 32 (two fit a CU at
// once).  Both plans sum every output in the same K order, so the choice
// changes speed only.  Measured: the 720p LR trunk (240 tiles) is 18% faster
// on the large tiles, the x8 network on a 1024 x 1024 image (64 tiles) 19%
// faster on the small ones.

void conv_launch_counts(int64_t* out, bool reset) {
  for (int i = 0; i < MRS_NUM_CONV_KINDS; ++i)
    out[i] = reset ? g_conv_launches[i].exchange(0) : g_conv_launches[i].load();
}

bool launch_res_block(const ConvArgs& a, const ConvArgs& b, hipStream_t st) {
  const auto fits = [](const ConvArgs& p) {
    return p.mode == VIEW_PLAIN && p.taps == 9 && p.cin_p == RB_C && p.kp == RB_KP &&
           p.cout == RB_C;
  };
  if (!fits(a) || !fits(b) || a.ca < RB_C || !a.relu || a.B != b.B || a.H != b.H ||
      a.W != b.W)
    return false;
  k_res_block<<<dim3((a.W + RB_T - 1) / RB_T, (a.H + RB_T - 1) / RB_T, a.B), RB_THREADS, 0,
                st>>>(a, b);
  count_conv(10);
  return true;
}

void launch_conv(const ConvArgs& a, int cout_p, hipStream_t st) {
  if (a.taps == 9 && a.mode != VIEW_CONCAT_UNSHUFFLE &&
      (a.mode != VIEW_PLAIN || a.ca >= a.cin_p)) {
    const int64_t tiles = (int64_t)((a.W + 15) / 16) * ((a.H + 15) / 16) * a.B;
    if (cout_p >= 64 && a.cin_p % 64 == 0 && tiles < conv_small_tiles() &&
        try_conv3_lds<64, 2, 8>(a, cout_p, cout_p / 32, st))
      return count_conv(0);
    if (cout_p >= 64) {
      if (try_conv3_lds<64, 4, 16>(a, cout_p, 1, st)) return count_conv(1);
      if (try_conv3_lds<16, 4, 16>(a, cout_p, 1, st)) return count_conv(2);
      if (try_conv3_lds<8, 4, 16>(a, cout_p, 1, st)) return count_conv(3);
    } else {
      if (try_conv3_lds<80, 1, 16>(a, cout_p, 1, st)) return count_conv(4);
      if (try_conv3_lds<64, 1, 16>(a, cout_p, 1, st)) return count_conv(5);
    }
  }
  const int64_t M = (int64_t)a.B * a.H * a.W;
  const unsigned gx = cdiv64(M, 128);
  if (cout_p >= 64) {
    k_conv<4><<<dim3(gx, cout_p / 64), 256, 0, st>>>(a);
    count_conv(6);
  } else {
    k_conv<1><<<dim3(gx, cout_p / 16), 256, 0, st>>>(a);
    count_conv(7);
  }
}

void launch_prep(const mrs_net* net, int64_t nhr, int64_t nlr, const float* hr, const float* aux,
                 const float* lr, uint16_t* xh, uint16_t* xl, hipStream_t st) {
  if (arch_has_layers(net->arch))
    k_prep_layers<<<cdiv64(nhr + nlr, 256), 256, 0, st>>>(
        nhr, nlr, hr, aux, net->in_layers, net->in_sumsq, 1.0f / (float)net->in_spp, lr, xh, xl);
  else
    k_prep<<<cdiv64(nhr + nlr, 256), 256, 0, st>>>(nhr, nlr, hr, aux, lr, xh, xl);
}

void launch_pack_all(const float* wm, const PackJob* jobs, int njobs, int64_t total,
                     uint16_t* packed, uint16_t* packed_t, hipStream_t st) {
  if (total > 0)
    k_pack_all<<<cdiv64(total, 256), 256, 0, st>>>(wm, jobs, njobs, total, packed, packed_t);
}

void launch_init(float* dst, const NetLayer& L, uint64_t seed, hipStream_t st) {
  const int64_t nw = (int64_t)L.cout * L.cin * L.k * L.k;
  const float bound = (float)(std::sqrt(6.0 / (double)(L.cin * L.k * L.k)) * L.init_scale);
  k_init<<<cdiv64(nw + L.cout, 256), 256, 0, st>>>(dst, nw, L.cout, (int64_t)L.w_off, bound,
                                                   (uint32_t)seed, (uint32_t)(seed >> 32));
}

}  // namespace mrs
