// Image metrics of the evaluation (paper Sec. 5): PSNR in sRGB (Eq. 3, peak 1)
// and RelMSE, with FP64 terms and a fixed-order two-pass reduction (results do
// not depend on scheduling).
#include "mrs_internal.hpp"

namespace mrs {
namespace {

constexpr int MB = 1024;  // partial sums (blocks) of the first pass

__device__ __forceinline__ double srgb(double l) {
  if (l <= 0.0) return 0.0;
  if (l <= 0.0031308) return 12.92 * l;
  if (l < 1.0) return 1.055 * pow(l, 1.0 / 2.4) - 0.055;
  return 1.0;
}

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sa, double* sb) {
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
}

__global__ __launch_bounds__(256) void k_metric_partial(const float* __restrict__ img,
                                                        const float* __restrict__ ref, int64_t n,
                                                        double lam1, double lam2,
                                                        double* __restrict__ part) {
  __shared__ double sa[256], sb[256];
  double se = 0.0, rel = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)MB * 256) {
    const double x = img[i], y = ref[i];
    const double d = srgb(x) - srgb(y);
    se += d * d;
    rel += lam1 * (x - y) * (x - y) / (y * y + lam2);
  }
  block_sum2(se, rel, sa, sb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = se;
    part[2 * blockIdx.x + 1] = rel;
  }
}

__global__ __launch_bounds__(256) void k_metric_final(const double* __restrict__ part, int64_t n,
                                                      double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  double se = 0.0, rel = 0.0;
  for (int b = threadIdx.x; b < MB; b += 256) {
    se += part[2 * b];
    rel += part[2 * b + 1];
  }
  block_sum2(se, rel, sa, sb);
  if (threadIdx.x == 0) {
    out[0] = se / (double)n;
    out[1] = rel / (double)n;
  }
}

double* g_part = nullptr;

}  // namespace

mrs_status image_metrics(const float* img, const float* ref, int64_t n, double lam1, double lam2,
                         double* out_dev, hipStream_t st) {
  if (!g_part) MRS_TRY_HIP(hipMalloc(&g_part, sizeof(double) * 2 * MB));
  k_metric_partial<<<MB, 256, 0, st>>>(img, ref, n, lam1, lam2, g_part);
  k_metric_final<<<1, 256, 0, st>>>(g_part, n, out_dev);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

}  // namespace mrs
