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

// 8 consecutive input channels [c, c+8) of tap `tap` around output pixel (b,y,x).
__device__ __forceinline__ bf16x8 load_chunk(const ConvArgs& p, int b, int y, int x, int tap,
                                             int c) {
  if (tap >= p.taps) return zero8();
  if (p.taps == 9) {
    y += tap / 3 - 1;
    x += tap % 3 - 1;
  }
  if (y < 0 || y >= p.H || x < 0 || x >= p.W) return zero8();
  const uint16_t* ptr;
  switch (p.mode) {
    case VIEW_PLAIN:
      ptr = p.a + ((size_t)(b * p.H + y) * p.W + x) * p.ca + c;
      break;
    case VIEW_CONCAT_UNSHUFFLE:  // [a (LR, ca ch), unshuffle_r(b (HR, cb ch))]
      if (c < p.ca) {
        ptr = p.a + ((size_t)(b * p.H + y) * p.W + x) * p.ca + c;
      } else {
        const int cc = c - p.ca;
        const int qq = cc / p.cb, ch = cc - qq * p.cb;
        const int hy = y * p.r + qq / p.r, hx = x * p.r + qq % p.r;
        ptr = p.b + ((size_t)(b * p.H * p.r + hy) * (p.W * p.r) + hx) * p.cb + ch;
      }
      break;
    default:  // VIEW_SHUFFLE_CONCAT: [shuffle_r(a (LR, ca = r^2 c0 ch)), b (HR, cb ch)]
      if (c < p.c0) {
        const int qq = (y % p.r) * p.r + (x % p.r);
        ptr = p.a + ((size_t)(b * (p.H / p.r) + y / p.r) * (p.W / p.r) + x / p.r) * p.ca +
              qq * p.c0 + c;
      } else {
        ptr = p.b + ((size_t)(b * p.H + y) * p.W + x) * p.cb + (c - p.c0);
      }
      break;
  }
  return ld8(ptr);
}

template <int NT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs p) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int M = p.B * p.H * p.W;
  const int m0 = (blockIdx.x * 4 + wave) * 32;
  if (m0 >= M) return;
  const int n0 = blockIdx.y * (NT * 16);
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
  f32x4 acc[2][NT];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int cpt = p.cin_p >> 3;  // 8-channel chunks per tap
  const uint16_t* wrow = p.w + (size_t)(n0 + li) * p.kp + kq * 8;
  for (int ks = 0; ks < p.kp; ks += 32) {
    const int q = (ks >> 3) + kq;
    const int tap = q / cpt;
    const int c = (q - tap * cpt) << 3;
    bf16x8 A[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) A[r] = pv[r] ? load_chunk(p, pb[r], py[r], px[r], tap, c) : zero8();
    bf16x8 Bv[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) Bv[j] = ld8(wrow + (size_t)j * 16 * p.kp + ks);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j)
        acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], Bv[j], acc[r][j], 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int n = n0 + j * 16 + li;
      if (n >= p.cout) continue;
      const float bias = p.bias[n];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + r * 16 + kq * 4 + v;
        if (m >= M) continue;
        float y = acc[r][j][v] + bias;
        if (p.relu) y = fmaxf(y, 0.0f);
        if (p.res) y = p.res[(size_t)m * p.cout + n] + p.res_scale * y;
        if (p.res2) y += p.res2[(size_t)m * p.cout + n];
        if (p.out_f) p.out_f[(size_t)m * p.out_f_stride + n] = y;
        if (p.out_h) p.out_h[(size_t)m * p.out_h_stride + n] = f2bf(y);
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

// Packed BF16 weights of one layer: wp[n][k], k = tap * cin_p + c; zero padding
// for c >= cin, tap >= taps, n >= cout.  Master layout [cout][cin][k][k].
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ wm, int cout, int cin,
                                              int ksz, int cin_p, int kp, int cout_p,
                                              uint16_t* __restrict__ wp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)cout_p * kp) return;
  const int n = (int)(i / kp), k = (int)(i % kp);
  const int tap = k / cin_p, c = k % cin_p;
  float v = 0.0f;
  if (n < cout && c < cin && tap < ksz * ksz) {
    const int ky = tap / ksz, kx = tap % ksz;
    v = wm[((size_t)(n * cin + c) * ksz + ky) * ksz + kx];
  }
  wp[i] = f2bf(v);
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

namespace {
inline unsigned cdiv64(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
}  // namespace

void launch_conv(const ConvArgs& a, int cout_p, hipStream_t st) {
  const int64_t M = (int64_t)a.B * a.H * a.W;
  const unsigned gx = cdiv64(M, 128);
  if (cout_p >= 64) {
    k_conv<4><<<dim3(gx, cout_p / 64), 256, 0, st>>>(a);
  } else {
    k_conv<1><<<dim3(gx, cout_p / 16), 256, 0, st>>>(a);
  }
}

void launch_prep(int64_t nhr, int64_t nlr, const float* hr, const float* aux, const float* lr,
                 uint16_t* xh, uint16_t* xl, hipStream_t st) {
  k_prep<<<cdiv64(nhr + nlr, 256), 256, 0, st>>>(nhr, nlr, hr, aux, lr, xh, xl);
}

void launch_pack(const float* wm, const NetLayer& L, uint16_t* wp, hipStream_t st) {
  k_pack<<<cdiv64((int64_t)L.cout_p * L.kp, 256), 256, 0, st>>>(wm, L.cout, L.cin, L.k, L.cin_p,
                                                                 L.kp, L.cout_p, wp);
}

void launch_init(float* dst, const NetLayer& L, uint64_t seed, hipStream_t st) {
  const int64_t nw = (int64_t)L.cout * L.cin * L.k * L.k;
  const float bound = (float)std::sqrt(6.0 / (double)(L.cin * L.k * L.k));
  k_init<<<cdiv64(nw + L.cout, 256), 256, 0, st>>>(dst, nw, L.cout, (int64_t)L.w_off, bound,
                                                   (uint32_t)seed, (uint32_t)(seed >> 32));
}

}  // namespace mrs
