// Linear BVH construction on the GPU (Karras, "Maximizing parallelism in the
// construction of BVHs, octrees, and k-d trees", HPG 2012).
//
//  1. centroid bounds (two-level min/max reduction)
//  2. 30-bit Morton code per triangle centroid, quantised in those bounds
//  3. stable LSD radix sort of (code, primitive) pairs, 8-bit digits; since the
//     primitives start in ascending order, the result is the order of the
//     unique 64-bit keys (code << 32 | primitive)
//  4. one internal node per adjacent key pair, its range and split found from
//     common-prefix lengths of the 64-bit keys (clz of xor)
//  5. leaf-to-root refit: each leaf walks up; the second thread to reach a
//     node (atomic visit counter) unions its children's boxes and continues.
//
// Node record (64 B): child boxes as 12 floats (left lo, left hi, right lo,
// right hi), then two child references (bit 31 = leaf) and 2 pad words.
#include "mrs_internal.hpp"
#include "devmath.hpp"

namespace mrs {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // keys per block

__device__ __forceinline__ f3 centroid(const float4* tri, int i) {
  f3 a = xyz(tri[3 * i]), b = xyz(tri[3 * i + 1]), c = xyz(tri[3 * i + 2]);
  return (a + b + c) * (1.0f / 3.0f);
}

__global__ __launch_bounds__(256) void k_bounds_partial(const float4* __restrict__ tri, int n,
                                                        float* __restrict__ part) {
  __shared__ float s[6][256];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    f3 c = centroid(tri, i);
    lo[0] = fminf(lo[0], c.x); lo[1] = fminf(lo[1], c.y); lo[2] = fminf(lo[2], c.z);
    hi[0] = fmaxf(hi[0], c.x); hi[1] = fmaxf(hi[1], c.y); hi[2] = fmaxf(hi[2], c.z);
  }
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = lo[a];
    s[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + w]);
        s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_bounds_final(const float* __restrict__ part, int nparts,
                                                     float* __restrict__ out) {
  if (threadIdx.x < 6) {
    const bool is_lo = threadIdx.x < 3;
    float v = is_lo ? INFINITY : -INFINITY;
    for (int b = 0; b < nparts; ++b) {
      float x = part[b * 6 + threadIdx.x];
      v = is_lo ? fminf(v, x) : fmaxf(v, x);
    }
    out[threadIdx.x] = v;
  }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v = (v * 0x00010001u) & 0xFF0000FFu;
  v = (v * 0x00000101u) & 0x0F00F00Fu;
  v = (v * 0x00000011u) & 0xC30C30C3u;
  v = (v * 0x00000005u) & 0x49249249u;
  return v;
}

__device__ __forceinline__ uint32_t quant10(float x, float lo, float ext) {
  float q = ext > 0.0f ? (x - lo) / ext : 0.0f;
  q = fminf(fmaxf(q * 1024.0f, 0.0f), 1023.0f);
  return (uint32_t)q;
}

__global__ __launch_bounds__(256) void k_morton(const float4* __restrict__ tri, int n,
                                                const float* __restrict__ bounds,
                                                uint32_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  f3 c = centroid(tri, i);
  uint32_t x = quant10(c.x, bounds[0], bounds[3] - bounds[0]);
  uint32_t y = quant10(c.y, bounds[1], bounds[4] - bounds[1]);
  uint32_t z = quant10(c.z, bounds[2], bounds[5] - bounds[2]);
  keys[i] = (spread10(x) << 2) | (spread10(y) << 1) | spread10(z);
  vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------- radix sort
// counts layout: digit-major, counts[d * nblocks + b]
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t* __restrict__ keys, int n,
                                                        int shift, int nblocks,
                                                        uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_ITEMS; ++k) {
    int i = base + k * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `len` counters with one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_rs_scan(uint32_t* __restrict__ counts, int len) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int seg = (len + 1023) / 1024;
  const int b = t * seg, e = min(len, b + seg);
  uint32_t sum = 0;
  for (int i = b; i < e; ++i) sum += counts[i];
  part[t] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;  // exclusive prefix of this segment
  for (int i = b; i < e; ++i) {
    uint32_t c = counts[i];
    counts[i] = run;
    run += c;
  }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Stable scatter: keys of a tile are ranked in tile order, 256 per round.  The
// rank among equal digits inside a wave comes from 8 ballots (one per digit
// bit); across the 4 waves of the block from per-wave digit counts in LDS.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, int n, int shift,
    int nblocks, const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[4][256];
  const int t = threadIdx.x;
  const int wave = t >> 6;
  base[t] = offsets[t * nblocks + blockIdx.x];
  for (int w = 0; w < 4; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const int tile = blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_ITEMS; ++k) {
    const int i = tile + k * RS_THREADS + t;
    const bool valid = i < n;
    uint32_t key = valid ? keys[i] : 0u;
    uint32_t val = valid ? vals[i] : 0u;
    uint32_t dig = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = lanes_below(peers);
    if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = base[dig] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][dig];
      if (off < (uint32_t)n) {  // always true for consistent counts; guards the write
        keys_out[off] = key;
        vals_out[off] = val;
      }
    }
    __syncthreads();
    base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    for (int w = 0; w < 4; ++w) wcnt[w][t] = 0;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- hierarchy
__device__ __forceinline__ int delta(const uint32_t* code, const uint32_t* prim, int n, int i,
                                     int j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = ((uint64_t)code[i] << 32) | prim[i];
  uint64_t b = ((uint64_t)code[j] << 32) | prim[j];
  return __clzll((long long)(a ^ b));
}

__global__ __launch_bounds__(256) void k_hierarchy(const uint32_t* __restrict__ code,
                                                   const uint32_t* __restrict__ prim, int n,
                                                   float4* __restrict__ nodes,
                                                   uint32_t* __restrict__ parent_int,
                                                   uint32_t* __restrict__ parent_leaf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n - 1) return;
  const int d = (delta(code, prim, n, i, i + 1) - delta(code, prim, n, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = delta(code, prim, n, i, i - d);
  int lmax = 2;
  while (delta(code, prim, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (delta(code, prim, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = delta(code, prim, n, i, j);
  int s = 0;
  int t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(code, prim, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int g = i + s * d + min(d, 0);
  const int lo = min(i, j), hi = max(i, j);
  if (g < lo || g + 1 > hi) return;  // cannot happen for unique keys; guards the writes
  uint32_t left, right;
  if (lo == g) {
    left = LEAF_BIT | (uint32_t)g;
    parent_leaf[g] = (uint32_t)i;
  } else {
    left = (uint32_t)g;
    parent_int[g] = (uint32_t)i;
  }
  if (hi == g + 1) {
    right = LEAF_BIT | (uint32_t)(g + 1);
    parent_leaf[g + 1] = (uint32_t)i;
  } else {
    right = (uint32_t)(g + 1);
    parent_int[g + 1] = (uint32_t)i;
  }
  nodes[4 * i + 3] = make_float4(__uint_as_float(left), __uint_as_float(right), 0.0f, 0.0f);
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Leaf records in leaf order, then the bottom-up refit.
__global__ __launch_bounds__(256) void k_leaves_refit(const float4* __restrict__ tri_src,
                                                      const uint32_t* __restrict__ leaf_prim,
                                                      int n, float4* __restrict__ leaf_tri,
                                                      float* __restrict__ nodes_f,
                                                      const uint32_t* __restrict__ parent_int,
                                                      const uint32_t* __restrict__ parent_leaf,
                                                      uint32_t* __restrict__ visits) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const uint32_t p = leaf_prim[k];
  const f3 v0 = xyz(tri_src[3 * p]), v1 = xyz(tri_src[3 * p + 1]), v2 = xyz(tri_src[3 * p + 2]);
  const f3 e1 = v1 - v0, e2 = v2 - v0;
  leaf_tri[3 * k + 0] = make_float4(v0.x, v0.y, v0.z, __uint_as_float(p));
  leaf_tri[3 * k + 1] = make_float4(e1.x, e1.y, e1.z, 0.0f);
  leaf_tri[3 * k + 2] = make_float4(e2.x, e2.y, e2.z, 0.0f);
  if (n < 2) return;
  float lo[3] = {fminf(v0.x, fminf(v1.x, v2.x)), fminf(v0.y, fminf(v1.y, v2.y)),
                 fminf(v0.z, fminf(v1.z, v2.z))};
  float hi[3] = {fmaxf(v0.x, fmaxf(v1.x, v2.x)), fmaxf(v0.y, fmaxf(v1.y, v2.y)),
                 fmaxf(v0.z, fmaxf(v1.z, v2.z))};
  uint32_t child = LEAF_BIT | (uint32_t)k;
  uint32_t node = parent_leaf[k];
  for (int guard = 0; guard < 2 * MAX_STACK + 2; ++guard) {
    if (node >= (uint32_t)(n - 1)) return;  // parents are always internal nodes
    float* nf = nodes_f + 16 * (size_t)node;
    const uint32_t left_ref = __float_as_uint(nf[12]);
    const int slot = (left_ref == child) ? 0 : 6;
    for (int a = 0; a < 3; ++a) {
      __hip_atomic_store(nf + slot + a, lo[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(nf + slot + 3 + a, hi[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t prev =
        __hip_atomic_fetch_add(visits + node, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == 0) return;  // the sibling subtree is not finished; its thread continues
    const int other = 6 - slot;
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __hip_atomic_load(nf + other + a, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
      hi[a] = fmaxf(hi[a], __hip_atomic_load(nf + other + 3 + a, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
    }
    if (node == 0) return;  // root: its box is not stored
    child = node;
    node = parent_int[node];
  }
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

mrs_status lbvh_build(mrs_scene* s, hipStream_t st) {
  const int n = s->ntris;
  s->bvh_built = false;
  if (n == 0) {
    s->root = 0;
    s->bvh_built = true;
    return MRS_OK;
  }
  // scratch: bounds partials, keys/vals ping-pong, counts, parents, visits
  const int nb = std::min(1024, cdiv(n, 256));
  const int rs_blocks = cdiv(n, RS_TILE);
  const size_t count_len = (size_t)256 * rs_blocks;
  size_t bytes = 0;
  auto carve = [&](size_t sz) {
    size_t off = bytes;
    bytes += (sz + 255) & ~(size_t)255;
    return off;
  };
  const size_t o_part = carve(sizeof(float) * 6 * nb);
  const size_t o_bounds = carve(sizeof(float) * 6);
  const size_t o_k0 = carve(sizeof(uint32_t) * n);
  const size_t o_v0 = carve(sizeof(uint32_t) * n);
  const size_t o_k1 = carve(sizeof(uint32_t) * n);
  const size_t o_v1 = carve(sizeof(uint32_t) * n);
  const size_t o_cnt = carve(sizeof(uint32_t) * count_len);
  const size_t o_pi = carve(sizeof(uint32_t) * n);
  const size_t o_pl = carve(sizeof(uint32_t) * n);
  const size_t o_vis = carve(sizeof(uint32_t) * n);
  char* scratch = nullptr;
  if (hipMalloc(&scratch, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_build_bvh: scratch allocation failed");
  }
  float* part = (float*)(scratch + o_part);
  float* bounds = (float*)(scratch + o_bounds);
  uint32_t* k0 = (uint32_t*)(scratch + o_k0);
  uint32_t* v0 = (uint32_t*)(scratch + o_v0);
  uint32_t* k1 = (uint32_t*)(scratch + o_k1);
  uint32_t* v1 = (uint32_t*)(scratch + o_v1);
  uint32_t* counts = (uint32_t*)(scratch + o_cnt);
  uint32_t* pint = (uint32_t*)(scratch + o_pi);
  uint32_t* pleaf = (uint32_t*)(scratch + o_pl);
  uint32_t* visits = (uint32_t*)(scratch + o_vis);

  k_bounds_partial<<<nb, 256, 0, st>>>(s->d_tri_src, n, part);
  k_bounds_final<<<1, 64, 0, st>>>(part, nb, bounds);
  k_morton<<<cdiv(n, 256), 256, 0, st>>>(s->d_tri_src, n, bounds, k0, v0);
  for (int shift = 0; shift < 32; shift += 8) {
    k_rs_hist<<<rs_blocks, RS_THREADS, 0, st>>>(k0, n, shift, rs_blocks, counts);
    k_rs_scan<<<1, 1024, 0, st>>>(counts, (int)count_len);
    k_rs_scatter<<<rs_blocks, RS_THREADS, 0, st>>>(k0, v0, n, shift, rs_blocks, counts, k1, v1);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  // 4 passes: the sorted data is back in the first buffers (k0/v0 after swaps)
  MRS_TRY_HIP(hipMemcpyAsync(s->d_morton, k0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
  MRS_TRY_HIP(
      hipMemcpyAsync(s->d_leaf_prim, v0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
  if (n >= 2) {
    k_hierarchy<<<cdiv(n - 1, 256), 256, 0, st>>>(s->d_morton, s->d_leaf_prim, n, s->d_nodes,
                                                  pint, pleaf);
    k_fill_u32<<<cdiv(n, 256), 256, 0, st>>>(visits, n, 0u);
  }
  k_leaves_refit<<<cdiv(n, 256), 256, 0, st>>>(s->d_tri_src, s->d_leaf_prim, n, s->d_leaf_tri,
                                               (float*)s->d_nodes, pint, pleaf, visits);
  MRS_TRY_HIP(hipGetLastError());
  // The scratch must outlive the kernels: wait, then free.
  MRS_TRY_HIP(hipStreamSynchronize(st));
  MRS_TRY_HIP(hipFree(scratch));
  s->root = n >= 2 ? 0u : LEAF_BIT;
  s->bvh_built = true;
  return MRS_OK;
}

}  // namespace mrs
