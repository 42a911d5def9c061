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
//  6. collapse to a four-wide BVH, top down one level per launch: a node
//     starts from its two binary children and twice opens the child of
//     largest surface area; binary subtrees of at most leaf_max triangles
//     become leaves (their leaf records are contiguous); nodes are then
//     renumbered densely in binary-node order.
//
// Binary node record (64 B): child boxes as 12 floats (left lo, left hi, right
// lo, right hi), two child references (bit 31 = leaf) and the node's range of
// leaf records (first, last).
//
// A second builder replaces steps 4-5 by agglomerative clustering over the
// Morton order (PLOC: Meister & Bittner, "Parallel Locally-Ordered Clustering
// for Bounding Volume Hierarchy Construction", IEEE TVCG 2018): every cluster
// finds, among the clusters within R places of it, the one whose union box has
// the smallest surface area; mutual nearest neighbours merge; the survivors are
// compacted in order; repeat until one cluster is left.  Ties are broken by a
// total order on cluster pairs, so some pair is always mutual and every round
// merges (identical boxes pair up with their neighbours, see pair_before).
// The tree is then laid out depth first: internal nodes numbered in
// preorder (root 0) and leaf records in leaf order, so every subtree's leaves
// are a contiguous range as the BVH4 collapse needs.  Its trees have a lower
// surface-area cost than the Morton-split tree (10-15% on the procedural
// scenes), hence fewer node visits and triangle tests per ray.
#include "mrs_internal.hpp"
#include "devmath.hpp"

namespace mrs {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // keys per block
constexpr int PLOC_RADIUS = 12;  // clusters searched on each side (fastest frame of 2..24)
constexpr int PLOC_MAX_ROUNDS = 256;

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
  nodes[4 * i + 3] = make_float4(__uint_as_float(left), __uint_as_float(right),
                                 __uint_as_float((uint32_t)lo), __uint_as_float((uint32_t)hi));
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

// ---------------------------------------------------------------- PLOC
constexpr uint32_t NO_PARENT = 0xffffffffu;

__device__ __forceinline__ float box_half_area(float4 lo, float4 hi) {
  const float dx = hi.x - lo.x, dy = hi.y - lo.y, dz = hi.z - lo.z;
  return dx * dy + dy * dz + dz * dx;
}

// Clusters start as the leaves in Morton order: reference LEAF_BIT | k.
__global__ __launch_bounds__(256) void k_ploc_init(const float4* __restrict__ tri_src,
                                                   const uint32_t* __restrict__ prim, int n,
                                                   uint32_t* __restrict__ cref,
                                                   float4* __restrict__ clo,
                                                   float4* __restrict__ chi) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const uint32_t p = prim[k];
  const f3 a = xyz(tri_src[3 * p]), b = xyz(tri_src[3 * p + 1]), c = xyz(tri_src[3 * p + 2]);
  cref[k] = LEAF_BIT | (uint32_t)k;
  clo[k] = make_float4(fminf(a.x, fminf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)),
                       fminf(a.z, fminf(b.z, c.z)), 0.0f);
  chi[k] = make_float4(fmaxf(a.x, fmaxf(b.x, c.x)), fmaxf(a.y, fmaxf(b.y, c.y)),
                       fmaxf(a.z, fmaxf(b.z, c.z)), 0.0f);
}

// Pair {c, j} before pair {c, b} in a total order of pairs: nearer pairs
// first, then pairs whose smaller member is even, then by smaller member (b < 0
// is no pair yet).  Among equal costs (equal boxes, regular grids) clusters
// thus pair up as (0, 1), (2, 3), ...: every cluster merges and the tree stays
// balanced, where a plain index order would merge one pair per round.
__device__ __forceinline__ bool pair_before(int c, int j, int b) {
  if (b < 0) return true;
  const int dj = abs(c - j), db = abs(c - b);
  if (dj != db) return dj < db;
  const int j0 = min(c, j), b0 = min(c, b);
  if ((j0 & 1) != (b0 & 1)) return (j0 & 1) == 0;
  return j0 < b0;
}

__global__ __launch_bounds__(256) void k_ploc_nn(int m, int radius,
                                                 const float4* __restrict__ clo,
                                                 const float4* __restrict__ chi,
                                                 int* __restrict__ nn) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  const float4 lo = clo[c], hi = chi[c];
  float best = INFINITY;
  int bj = -1;
  const int j0 = max(0, c - radius), j1 = min(m - 1, c + radius);
  for (int j = j0; j <= j1; ++j) {
    if (j == c) continue;
    const float4 l2 = clo[j], h2 = chi[j];
    const float a = box_half_area(
        make_float4(fminf(lo.x, l2.x), fminf(lo.y, l2.y), fminf(lo.z, l2.z), 0.0f),
        make_float4(fmaxf(hi.x, h2.x), fmaxf(hi.y, h2.y), fmaxf(hi.z, h2.z), 0.0f));
    if (a < best || (a == best && pair_before(c, j, bj))) {
      best = a;
      bj = j;
    }
  }
  nn[c] = bj;
}

// Mutual nearest neighbours c < j merge into a new internal node (in place of
// c; j is dropped).  The node's record gets the two child boxes and references.
__global__ __launch_bounds__(256) void k_ploc_merge(int m, int nint, const int* __restrict__ nn,
                                                    uint32_t* __restrict__ cref,
                                                    float4* __restrict__ clo,
                                                    float4* __restrict__ chi,
                                                    float* __restrict__ tnodes,
                                                    uint32_t* __restrict__ tcount,
                                                    uint32_t* __restrict__ keep) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  const int j = nn[c];
  const bool mutual = j >= 0 && j < m && nn[j] == c;
  keep[c] = (mutual && c > j) ? 0u : 1u;
  if (!mutual || c > j) return;
  const uint32_t t = atomicAdd(tcount, 1u);
  if (t >= (uint32_t)nint) return;  // cannot happen: n leaves make n - 1 merges
  const float4 l1 = clo[c], h1 = chi[c], l2 = clo[j], h2 = chi[j];
  float* o = tnodes + 16 * (size_t)t;
  o[0] = l1.x; o[1] = l1.y; o[2] = l1.z; o[3] = h1.x; o[4] = h1.y; o[5] = h1.z;
  o[6] = l2.x; o[7] = l2.y; o[8] = l2.z; o[9] = h2.x; o[10] = h2.y; o[11] = h2.z;
  o[12] = __uint_as_float(cref[c]);
  o[13] = __uint_as_float(cref[j]);
  o[14] = o[15] = 0.0f;
  cref[c] = t;
  clo[c] = make_float4(fminf(l1.x, l2.x), fminf(l1.y, l2.y), fminf(l1.z, l2.z), 0.0f);
  chi[c] = make_float4(fmaxf(h1.x, h2.x), fmaxf(h1.y, h2.y), fmaxf(h1.z, h2.z), 0.0f);
}

__global__ __launch_bounds__(256) void k_ploc_count(int m, const uint32_t* __restrict__ keep,
                                                    uint32_t* __restrict__ bcount) {
  __shared__ uint32_t wc[4];
  const int c = blockIdx.x * 256 + threadIdx.x;
  const uint64_t b = __ballot(c < m && keep[c]);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) bcount[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// Kept clusters in order into the other arrays (boff: exclusive block offsets);
// the last cluster's thread writes the new count.
__global__ __launch_bounds__(256) void k_ploc_scatter(
    int m, const uint32_t* __restrict__ keep, const uint32_t* __restrict__ boff,
    const uint32_t* __restrict__ cref, const float4* __restrict__ clo,
    const float4* __restrict__ chi, uint32_t* __restrict__ cref2, float4* __restrict__ clo2,
    float4* __restrict__ chi2, uint32_t* __restrict__ mcount) {
  __shared__ uint32_t wc[4];
  const int c = blockIdx.x * 256 + threadIdx.x;
  const bool k = c < m && keep[c];
  const uint64_t b = __ballot(k);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t pos = boff[blockIdx.x] + lanes_below(b);
  for (int v = 0; v < w; ++v) pos += wc[v];
  if (k && pos < (uint32_t)m) {
    cref2[pos] = cref[c];
    clo2[pos] = clo[c];
    chi2[pos] = chi[c];
  }
  if (c == m - 1) *mcount = pos + (k ? 1u : 0u);
}

// Parent of every node and leaf: (parent << 1) | side.
__global__ __launch_bounds__(256) void k_ploc_parents(int nint, const float* __restrict__ tnodes,
                                                      uint32_t* __restrict__ par_int,
                                                      uint32_t* __restrict__ par_leaf, int n) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nint) return;
  for (int side = 0; side < 2; ++side) {
    const uint32_t r = __float_as_uint(tnodes[16 * (size_t)t + 12 + side]);
    const uint32_t v = ((uint32_t)t << 1) | (uint32_t)side;
    if (r & LEAF_BIT) {
      if ((r & ~LEAF_BIT) < (uint32_t)n) par_leaf[r & ~LEAF_BIT] = v;
    } else if (r < (uint32_t)nint) {
      par_int[r] = v;
    }
  }
}

// Leaf counts of each node's two subtrees (sz2[2t + side]), bottom up: every
// leaf walks up; the second arrival at a node (visit counter) continues.
__global__ __launch_bounds__(256) void k_ploc_sizes(int n, const uint32_t* __restrict__ par_int,
                                                    const uint32_t* __restrict__ par_leaf,
                                                    uint32_t* __restrict__ sz2,
                                                    uint32_t* __restrict__ visits,
                                                    uint32_t* __restrict__ deep,
                                                    uint32_t* __restrict__ bad) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  uint32_t size = 1;
  uint32_t x = par_leaf[k];
  for (int guard = 0; guard < 4 * MAX_STACK; ++guard) {
    if (x == NO_PARENT) return;
    const uint32_t p = x >> 1, side = x & 1u;
    if (p >= (uint32_t)(n - 1)) {  // cannot happen for a tree
      atomicOr(bad, 1u);
      return;
    }
    __hip_atomic_store(sz2 + 2 * p + side, size, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t prev =
        __hip_atomic_fetch_add(visits + p, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == 0) return;  // the sibling subtree is not finished; its thread continues
    size += __hip_atomic_load(sz2 + 2 * p + (1u - side), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    x = par_int[p];
  }
  atomicMax(deep, (uint32_t)(4 * MAX_STACK));  // deeper than the walk's bound: too deep
}

// Depth-first layout, each node and leaf walking up to the root: a left child
// comes right after its parent in preorder and shares its first leaf; a right
// child follows the left subtree (its leaf count L): preorder + L, first leaf + L.
__global__ __launch_bounds__(256) void k_ploc_order(int n, int nint,
                                                    const uint32_t* __restrict__ par_int,
                                                    const uint32_t* __restrict__ par_leaf,
                                                    const uint32_t* __restrict__ sz2,
                                                    uint32_t* __restrict__ pre_int,
                                                    uint32_t* __restrict__ first_int,
                                                    uint32_t* __restrict__ first_leaf,
                                                    uint32_t* __restrict__ depth_max,
                                                    uint32_t* __restrict__ bad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nint + n) return;
  uint32_t x = i < nint ? par_int[i] : par_leaf[i - nint];
  uint32_t pre = 0, first = 0, depth = 0;
  for (; x != NO_PARENT; ++depth) {
    if (depth >= 4 * MAX_STACK) {  // too deep (the caller falls back)
      atomicMax(depth_max, depth);
      return;
    }
    const uint32_t p = x >> 1;
    if (p >= (uint32_t)nint) {  // cannot happen for a tree
      atomicOr(bad, 1u);
      return;
    }
    if (x & 1u) {
      const uint32_t L = sz2[2 * p];
      pre += L;
      first += L;
    } else {
      pre += 1;
    }
    x = par_int[p];
  }
  if (i < nint) {
    pre_int[i] = pre;
    first_int[i] = first;
  } else {
    first_leaf[i - nint] = first;
  }
  atomicMax(depth_max, depth);
}

// Final binary records: temporary node t goes to its preorder place, with its
// references and leaf range in the final numbering.
__global__ __launch_bounds__(256) void k_ploc_emit(int nint, int n, const float* __restrict__ tnodes,
                                                   const uint32_t* __restrict__ pre_int,
                                                   const uint32_t* __restrict__ first_int,
                                                   const uint32_t* __restrict__ first_leaf,
                                                   const uint32_t* __restrict__ sz2,
                                                   float* __restrict__ nodes_f) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nint) return;
  const uint32_t d = pre_int[t];
  if (d >= (uint32_t)nint) return;  // cannot happen for a tree
  const float* src = tnodes + 16 * (size_t)t;
  float* o = nodes_f + 16 * (size_t)d;
  for (int a = 0; a < 12; ++a) o[a] = src[a];
  for (int side = 0; side < 2; ++side) {
    const uint32_t r = __float_as_uint(src[12 + side]);
    uint32_t f;
    if (r & LEAF_BIT) f = LEAF_BIT | first_leaf[min(r & ~LEAF_BIT, (uint32_t)n - 1)];
    else f = pre_int[min(r, (uint32_t)nint - 1)];
    o[12 + side] = __uint_as_float(f);
  }
  const uint32_t first = first_int[t];
  o[14] = __uint_as_float(first);
  o[15] = __uint_as_float(first + sz2[2 * t] + sz2[2 * t + 1] - 1u);
}

// Morton position k -> leaf position first_leaf[k]: primitives and codes in
// leaf order.
__global__ __launch_bounds__(256) void k_ploc_leaves(int n, const uint32_t* __restrict__ prim,
                                                     const uint32_t* __restrict__ code,
                                                     const uint32_t* __restrict__ first_leaf,
                                                     uint32_t* __restrict__ leaf_prim,
                                                     uint32_t* __restrict__ leaf_code) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const uint32_t pos = first_leaf[k];
  if (pos >= (uint32_t)n) return;  // cannot happen for a tree
  leaf_prim[pos] = prim[k];
  leaf_code[pos] = code[k];
}

// Leaf records (v0, primitive id) (e1) (e2) in leaf order.
__global__ __launch_bounds__(256) void k_leaf_records(const float4* __restrict__ tri_src,
                                                      const uint32_t* __restrict__ leaf_prim,
                                                      int n, float4* __restrict__ leaf_tri) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const uint32_t p = leaf_prim[k];
  if (p >= (uint32_t)n) return;  // cannot happen: leaf_prim is a permutation
  const f3 v0 = xyz(tri_src[3 * p]), v1 = xyz(tri_src[3 * p + 1]), v2 = xyz(tri_src[3 * p + 2]);
  const f3 e1 = v1 - v0, e2 = v2 - v0;
  leaf_tri[3 * k + 0] = make_float4(v0.x, v0.y, v0.z, __uint_as_float(p));
  leaf_tri[3 * k + 1] = make_float4(e1.x, e1.y, e1.z, 0.0f);
  leaf_tri[3 * k + 2] = make_float4(e2.x, e2.y, e2.z, 0.0f);
}

// ---------------------------------------------------------------- BVH4 collapse
struct Cand {
  uint32_t ref;
  float lo[3], hi[3];
};

__device__ __forceinline__ void binary_children(const float* __restrict__ nf, Cand& l, Cand& r) {
  for (int a = 0; a < 3; ++a) {
    l.lo[a] = nf[a];
    l.hi[a] = nf[3 + a];
    r.lo[a] = nf[6 + a];
    r.hi[a] = nf[9 + a];
  }
  l.ref = __float_as_uint(nf[12]);
  r.ref = __float_as_uint(nf[13]);
}

__device__ __forceinline__ float half_area(const Cand& c) {
  const float dx = c.hi[0] - c.lo[0], dy = c.hi[1] - c.lo[1], dz = c.hi[2] - c.lo[2];
  return dx * dy + dy * dz + dz * dx;
}

// leaf-record range of a binary reference
__device__ __forceinline__ void ref_range(const float* __restrict__ nodes_f, uint32_t ref,
                                          uint32_t& first, uint32_t& last) {
  if (ref & LEAF_BIT) {
    first = last = ref & ~LEAF_BIT;
  } else {
    first = __float_as_uint(nodes_f[16 * (size_t)ref + 14]);
    last = __float_as_uint(nodes_f[16 * (size_t)ref + 15]);
  }
}

// One level: each queued binary node b becomes BVH4 node b (sparse numbering).
__global__ __launch_bounds__(256) void k_collapse(const float* __restrict__ nodes_f,
                                                  const uint32_t* __restrict__ q_in,
                                                  const uint32_t* __restrict__ cnt_in,
                                                  uint32_t* __restrict__ q_out,
                                                  uint32_t* __restrict__ cnt_out,
                                                  float4* __restrict__ sparse4,
                                                  uint32_t* __restrict__ is4, int leaf_max) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= *cnt_in) return;
  const uint32_t b = q_in[i];
  Cand c[4];
  binary_children(nodes_f + 16 * (size_t)b, c[0], c[1]);
  int nc = 2;
  for (int open = 0; open < 2; ++open) {
    int best = -1;
    float best_area = -1.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= nc || (c[k].ref & LEAF_BIT)) continue;
      uint32_t f, l;
      ref_range(nodes_f, c[k].ref, f, l);
      if (l - f + 1 <= (uint32_t)leaf_max) continue;
      const float a = half_area(c[k]);
      if (a > best_area) {
        best_area = a;
        best = k;
      }
    }
    if (best < 0) break;
    Cand l, r;
    uint32_t opened = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k == best) opened = c[k].ref;
    binary_children(nodes_f + 16 * (size_t)opened, l, r);
    // c[best] <- l, c[best + 1] <- r, later children shift right by one
#pragma unroll
    for (int k = 3; k >= 1; --k)
      if (k > best + 1 && k <= nc) c[k] = c[k - 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k == best) c[k] = l;
      if (k == best + 1) c[k] = r;
    }
    ++nc;
  }
  float box[6][4];
  uint32_t refs[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < nc) {
      uint32_t f, l;
      ref_range(nodes_f, c[k].ref, f, l);
      if ((c[k].ref & LEAF_BIT) || l - f + 1 <= (uint32_t)leaf_max) {
        refs[k] = leaf4_ref(f, l - f + 1);
      } else {
        refs[k] = c[k].ref;
        q_out[atomicAdd(cnt_out, 1u)] = c[k].ref;
      }
      for (int a = 0; a < 3; ++a) {
        box[a][k] = c[k].lo[a];
        box[3 + a][k] = c[k].hi[a];
      }
    } else {
      refs[k] = EMPTY4;
      for (int a = 0; a < 3; ++a) {
        box[a][k] = INFINITY;
        box[3 + a][k] = -INFINITY;
      }
    }
  }
  float4* o = sparse4 + 8 * (size_t)b;
  for (int a = 0; a < 6; ++a) o[a] = make_float4(box[a][0], box[a][1], box[a][2], box[a][3]);
  o[6] = make_float4(__uint_as_float(refs[0]), __uint_as_float(refs[1]),
                     __uint_as_float(refs[2]), __uint_as_float(refs[3]));
  o[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  is4[b] = 1u;
}

// Dense renumbering (binary-node order): node b moves to idx[b]; internal
// references are renumbered the same way.
__global__ __launch_bounds__(256) void k_compact4(const float4* __restrict__ sparse4,
                                                  const uint32_t* __restrict__ is4,
                                                  const uint32_t* __restrict__ idx, int nint,
                                                  float4* __restrict__ dense4) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nint || !is4[b]) return;
  const float4* src = sparse4 + 8 * (size_t)b;
  float4* dst = dense4 + 8 * (size_t)idx[b];
  for (int a = 0; a < 6; ++a) dst[a] = src[a];
  const float4 r = src[6];
  uint32_t refs[4] = {__float_as_uint(r.x), __float_as_uint(r.y), __float_as_uint(r.z),
                      __float_as_uint(r.w)};
  for (int k = 0; k < 4; ++k)
    if (refs[k] != EMPTY4 && !(refs[k] & LEAF_BIT)) refs[k] = idx[refs[k]];
  dst[6] = make_float4(__uint_as_float(refs[0]), __uint_as_float(refs[1]),
                       __uint_as_float(refs[2]), __uint_as_float(refs[3]));
  dst[7] = src[7];
}

// Quantized copy of a BVH4 node (64 bytes, 4 float4): the node's box origin p
// (minus a margin) and per-axis power-of-two steps s = 2^e, then each child's
// box as 8-bit steps from p, rounded outward, and the child references:
//   [0] p.x, p.y, p.z, bits(biased e_x | e_y << 8 | e_z << 16)
//   [1] lo_x, lo_y, lo_z, hi_x  (one byte per child: byte c = child c)
//   [2] hi_y, hi_z, 0, 0
//   [3] child references (as in the full node)
// Every quantized child box contains the exact one with a margin of at least
// m = 2^-18 max(|node coordinates|, |scene coordinates|) on every side, so the
// traversal's FP32 rounding never culls a box the full node would keep.
__global__ __launch_bounds__(256) void k_quantize4(const float4* __restrict__ nodes4, int count,
                                                   float4* __restrict__ q4) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float4* nd = nodes4 + 8 * (size_t)i;
  const float4* root = nodes4;
  const float4 rf = nd[6];
  const uint32_t ref[4] = {__float_as_uint(rf.x), __float_as_uint(rf.y), __float_as_uint(rf.z),
                           __float_as_uint(rf.w)};
  auto comp = [](const float4& v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; };
  double scene = 0.0;  // largest coordinate magnitude of the scene (the root's child boxes)
  {
    const uint32_t rr[4] = {__float_as_uint(root[6].x), __float_as_uint(root[6].y),
                            __float_as_uint(root[6].z), __float_as_uint(root[6].w)};
    for (int c = 0; c < 4; ++c)
      if (rr[c] != EMPTY4)
        for (int a = 0; a < 6; ++a) scene = fmax(scene, fabs((double)comp(root[a], c)));
  }
  float P[3];
  uint32_t E = 0, qlo[3] = {0u, 0u, 0u}, qhi[3] = {0u, 0u, 0u};
  for (int a = 0; a < 3; ++a) {
    double lo = INFINITY, hi = -INFINITY, mag = scene;
    for (int c = 0; c < 4; ++c) {
      if (ref[c] == EMPTY4) continue;
      const double l = comp(nd[a], c), h = comp(nd[3 + a], c);
      lo = fmin(lo, l);
      hi = fmax(hi, h);
      mag = fmax(mag, fmax(fabs(l), fabs(h)));
    }
    if (!(lo <= hi)) lo = hi = 0.0;  // no child (cannot happen in a built tree)
    const double m = ldexp(fmax(mag, 1e-30), -18);
    // origin: an FP32 value at or below lo - m
    float p = (float)(lo - m);
    if ((double)p > lo - m) p = nextafterf(p, -INFINITY);
    // step: the smallest power of two with 255 steps covering [p, hi + m]
    const double need = (hi + m - (double)p) / 255.0;
    int e;
    (void)frexp(fmax(need, 1e-37), &e);  // need <= 2^e
    e = max(-126, min(127, e));
    const double sc = ldexp(1.0, e);
    P[a] = p;
    E |= (uint32_t)(e + 127) << (8 * a);
    for (int c = 0; c < 4; ++c) {
      uint32_t ql = 0u, qh = 0u;
      if (ref[c] != EMPTY4) {
        const double l = comp(nd[a], c) - m, h = comp(nd[3 + a], c) + m;
        int lq = (int)floor((l - (double)p) / sc), hq = (int)ceil((h - (double)p) / sc);
        lq = max(0, min(255, lq));
        hq = max(0, min(255, hq));
        while (lq > 0 && (double)p + lq * sc > l) --lq;   // exact in FP64
        while (hq < 255 && (double)p + hq * sc < h) ++hq;
        ql = (uint32_t)lq;
        qh = (uint32_t)hq;
      }
      qlo[a] |= ql << (8 * c);
      qhi[a] |= qh << (8 * c);
    }
  }
  float4* o = q4 + 4 * (size_t)i;
  o[0] = make_float4(P[0], P[1], P[2], __uint_as_float(E));
  o[1] = make_float4(__uint_as_float(qlo[0]), __uint_as_float(qlo[1]), __uint_as_float(qlo[2]),
                     __uint_as_float(qhi[0]));
  o[2] = make_float4(__uint_as_float(qhi[1]), __uint_as_float(qhi[2]), 0.0f, 0.0f);
  o[3] = rf;
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// Top-down collapse of the binary tree (one launch per BVH4 level; the level
// size is read back to size the next launch), then dense renumbering.
mrs_status collapse4(mrs_scene* s, hipStream_t st, int leaf_max, char* scratch, size_t o_q0,
                     size_t o_q1, size_t o_qc, size_t o_is4, size_t o_idx, size_t o_sp4) {
  const int n = s->ntris;
  uint32_t* q[2] = {(uint32_t*)(scratch + o_q0), (uint32_t*)(scratch + o_q1)};
  uint32_t* qc = (uint32_t*)(scratch + o_qc);
  uint32_t* is4 = (uint32_t*)(scratch + o_is4);
  uint32_t* idx = (uint32_t*)(scratch + o_idx);
  float4* sparse4 = (float4*)(scratch + o_sp4);
  k_fill_u32<<<cdiv(n - 1, 256), 256, 0, st>>>(is4, n - 1, 0u);
  k_fill_u32<<<1, 256, 0, st>>>(q[0], 1, 0u);  // the root is the one item of level 0
  k_fill_u32<<<1, 256, 0, st>>>(qc, 1, 1u);
  uint32_t items = 1;
  int cur = 0;
  for (int level = 0; items > 0; ++level) {
    if (level > 4 * MAX_STACK) return fail(MRS_ERR_DEVICE, "mrs_build_bvh: BVH4 collapse does not end");
    k_fill_u32<<<1, 256, 0, st>>>(qc + (1 - cur), 1, 0u);
    k_collapse<<<cdiv(items, 256), 256, 0, st>>>((const float*)s->d_nodes, q[cur], qc + cur,
                                                  q[1 - cur], qc + (1 - cur), sparse4, is4,
                                                  leaf_max);
    MRS_TRY_HIP(hipGetLastError());
    MRS_TRY_HIP(hipMemcpyAsync(&items, qc + (1 - cur), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MRS_TRY_HIP(hipStreamSynchronize(st));
    cur = 1 - cur;
  }
  MRS_TRY_HIP(hipMemcpyAsync(idx, is4, sizeof(uint32_t) * (n - 1), hipMemcpyDeviceToDevice, st));
  k_rs_scan<<<1, 1024, 0, st>>>(idx, n - 1);
  uint32_t last_idx = 0, last_is = 0;
  MRS_TRY_HIP(hipMemcpyAsync(&last_idx, idx + (n - 2), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipMemcpyAsync(&last_is, is4 + (n - 2), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  const uint32_t count4 = last_idx + last_is;
  if (s->d_nodes4) {
    (void)hipFree(s->d_nodes4);
    s->d_nodes4 = nullptr;
  }
  if (hipMalloc(&s->d_nodes4, sizeof(float4) * 8 * (size_t)count4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_build_bvh: BVH4 allocation failed");
  }
  k_compact4<<<cdiv(n - 1, 256), 256, 0, st>>>(sparse4, is4, idx, n - 1, s->d_nodes4);
  MRS_TRY_HIP(hipGetLastError());
  if (s->d_nodes4q) {
    (void)hipFree(s->d_nodes4q);
    s->d_nodes4q = nullptr;
  }
  if (hipMalloc(&s->d_nodes4q, sizeof(float4) * 4 * (size_t)count4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_build_bvh: quantized BVH4 allocation failed");
  }
  k_quantize4<<<cdiv(count4, 256), 256, 0, st>>>(s->d_nodes4, (int)count4, s->d_nodes4q);
  MRS_TRY_HIP(hipGetLastError());
  s->count4 = count4;
  s->root4 = 0u;  // binary root 0 is the first BVH4 node
  return MRS_OK;
}

// PLOC over the Morton-sorted primitives (code, prim): binary records into
// s->d_nodes (preorder, root 0), primitives and codes in leaf order into
// s->d_leaf_prim / s->d_morton, leaf records into s->d_leaf_tri.  *used is
// false (and nothing of the scene written) when the tree would be deeper than
// the Morton-split tree may be (64 levels): the caller builds that one instead.
mrs_status ploc_build(mrs_scene* s, hipStream_t st, const uint32_t* code, const uint32_t* prim,
                      int radius, bool* used) {
  *used = false;
  const int n = s->ntris, nint = n - 1;
  const int nb = cdiv(n, 256);
  size_t bytes = 0;
  auto carve = [&](size_t sz) {
    size_t off = bytes;
    bytes += (sz + 255) & ~(size_t)255;
    return off;
  };
  size_t o_ref[2], o_lo[2], o_hi[2];
  for (int b = 0; b < 2; ++b) {
    o_ref[b] = carve(sizeof(uint32_t) * n);
    o_lo[b] = carve(sizeof(float4) * n);
    o_hi[b] = carve(sizeof(float4) * n);
  }
  const size_t o_nn = carve(sizeof(int) * n);
  const size_t o_keep = carve(sizeof(uint32_t) * n);
  const size_t o_boff = carve(sizeof(uint32_t) * nb);
  const size_t o_tn = carve(sizeof(float) * 16 * (size_t)nint);
  const size_t o_pi = carve(sizeof(uint32_t) * nint);
  const size_t o_pl = carve(sizeof(uint32_t) * n);
  const size_t o_sz = carve(sizeof(uint32_t) * 2 * (size_t)nint);
  const size_t o_vis = carve(sizeof(uint32_t) * nint);
  const size_t o_pre = carve(sizeof(uint32_t) * nint);
  const size_t o_fi = carve(sizeof(uint32_t) * nint);
  const size_t o_fl = carve(sizeof(uint32_t) * n);
  const size_t o_ctr = carve(sizeof(uint32_t) * 4);  // merges, count, depth, bad
  char* scratch = nullptr;
  if (hipMalloc(&scratch, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_build_bvh: clustering scratch allocation failed");
  }
  uint32_t* cref[2] = {(uint32_t*)(scratch + o_ref[0]), (uint32_t*)(scratch + o_ref[1])};
  float4* clo[2] = {(float4*)(scratch + o_lo[0]), (float4*)(scratch + o_lo[1])};
  float4* chi[2] = {(float4*)(scratch + o_hi[0]), (float4*)(scratch + o_hi[1])};
  int* nn = (int*)(scratch + o_nn);
  uint32_t* keep = (uint32_t*)(scratch + o_keep);
  uint32_t* boff = (uint32_t*)(scratch + o_boff);
  float* tnodes = (float*)(scratch + o_tn);
  uint32_t* par_int = (uint32_t*)(scratch + o_pi);
  uint32_t* par_leaf = (uint32_t*)(scratch + o_pl);
  uint32_t* sz2 = (uint32_t*)(scratch + o_sz);
  uint32_t* visits = (uint32_t*)(scratch + o_vis);
  uint32_t* pre_int = (uint32_t*)(scratch + o_pre);
  uint32_t* first_int = (uint32_t*)(scratch + o_fi);
  uint32_t* first_leaf = (uint32_t*)(scratch + o_fl);
  uint32_t* ctr = (uint32_t*)(scratch + o_ctr);
  mrs_status rc = MRS_OK;
  auto run = [&]() -> mrs_status {
    k_fill_u32<<<1, 256, 0, st>>>(ctr, 4, 0u);
    k_ploc_init<<<nb, 256, 0, st>>>(s->d_tri_src, prim, n, cref[0], clo[0], chi[0]);
    int cur = 0;
    uint32_t m = (uint32_t)n;
    for (int round = 0; m > 1; ++round) {
      // a healthy build takes 50-70 rounds; this many means chains (deep trees)
      if (round >= PLOC_MAX_ROUNDS) return MRS_OK;  // the caller falls back
      const int mb = cdiv(m, 256);
      k_ploc_nn<<<mb, 256, 0, st>>>((int)m, radius, clo[cur], chi[cur], nn);
      k_ploc_merge<<<mb, 256, 0, st>>>((int)m, nint, nn, cref[cur], clo[cur], chi[cur], tnodes,
                                       ctr, keep);
      k_ploc_count<<<mb, 256, 0, st>>>((int)m, keep, boff);
      k_rs_scan<<<1, 1024, 0, st>>>(boff, mb);
      k_ploc_scatter<<<mb, 256, 0, st>>>((int)m, keep, boff, cref[cur], clo[cur], chi[cur],
                                         cref[1 - cur], clo[1 - cur], chi[1 - cur], ctr + 1);
      MRS_TRY_HIP(hipGetLastError());
      uint32_t m2 = 0;
      MRS_TRY_HIP(hipMemcpyAsync(&m2, ctr + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      MRS_TRY_HIP(hipStreamSynchronize(st));
      if (m2 >= m || m2 == 0)
        return fail(MRS_ERR_DEVICE, "mrs_build_bvh: a clustering round merged nothing");
      m = m2;
      cur = 1 - cur;
    }
    uint32_t root = 0, merges = 0;
    MRS_TRY_HIP(hipMemcpyAsync(&root, cref[cur], sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MRS_TRY_HIP(hipMemcpyAsync(&merges, ctr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MRS_TRY_HIP(hipStreamSynchronize(st));
    if (merges != (uint32_t)nint || (root & LEAF_BIT) || root >= (uint32_t)nint)
      return fail(MRS_ERR_DEVICE, "mrs_build_bvh: clustering did not make one tree");
    k_fill_u32<<<cdiv(nint, 256), 256, 0, st>>>(par_int, nint, NO_PARENT);
    k_fill_u32<<<nb, 256, 0, st>>>(par_leaf, n, NO_PARENT);
    k_fill_u32<<<cdiv(nint, 256), 256, 0, st>>>(visits, nint, 0u);
    k_ploc_parents<<<cdiv(nint, 256), 256, 0, st>>>(nint, tnodes, par_int, par_leaf, n);
    k_ploc_sizes<<<nb, 256, 0, st>>>(n, par_int, par_leaf, sz2, visits, ctr + 2, ctr + 3);
    k_ploc_order<<<cdiv(nint + n, 256), 256, 0, st>>>(n, nint, par_int, par_leaf, sz2, pre_int,
                                                      first_int, first_leaf, ctr + 2, ctr + 3);
    MRS_TRY_HIP(hipGetLastError());
    uint32_t dm[2] = {0, 0};
    MRS_TRY_HIP(hipMemcpyAsync(dm, ctr + 2, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MRS_TRY_HIP(hipStreamSynchronize(st));
    if (dm[1]) return fail(MRS_ERR_DEVICE, "mrs_build_bvh: clustered tree is malformed");
    if (dm[0] > (uint32_t)MAX_STACK) return MRS_OK;  // too deep: the caller falls back
    k_ploc_emit<<<cdiv(nint, 256), 256, 0, st>>>(nint, n, tnodes, pre_int, first_int,
                                                 first_leaf, sz2, (float*)s->d_nodes);
    k_ploc_leaves<<<nb, 256, 0, st>>>(n, prim, code, first_leaf, s->d_leaf_prim, s->d_morton);
    k_leaf_records<<<nb, 256, 0, st>>>(s->d_tri_src, s->d_leaf_prim, n, s->d_leaf_tri);
    MRS_TRY_HIP(hipGetLastError());
    *used = true;
    return MRS_OK;
  };
  rc = run();
  // The scratch must outlive the kernels: wait, then free.
  (void)hipStreamSynchronize(st);
  (void)hipFree(scratch);
  return rc;
}

}  // namespace

mrs_status lbvh_build(mrs_scene* s, hipStream_t st, int leaf_max, int builder) {
  const int n = s->ntris;
  s->bvh_built = false;
  s->leaf_max = leaf_max;
  if (n == 0) {
    s->root = 0;
    s->root4 = EMPTY4;
    s->count4 = 0;
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
  const size_t o_q0 = carve(sizeof(uint32_t) * n);
  const size_t o_q1 = carve(sizeof(uint32_t) * n);
  const size_t o_qc = carve(sizeof(uint32_t) * 2);
  const size_t o_is4 = carve(sizeof(uint32_t) * n);
  const size_t o_idx = carve(sizeof(uint32_t) * n);
  const size_t o_sp4 = carve(sizeof(float4) * 8 * (size_t)std::max(n - 1, 1));
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
  bool clustered = false;
  mrs_status rc = MRS_OK;
  if (builder == MRS_BVH_PLOC && n >= 2) {
    rc = ploc_build(s, st, k0, v0, PLOC_RADIUS, &clustered);
    if (rc != MRS_OK) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(scratch);
      return rc;
    }
  }
  if (!clustered) {
    MRS_TRY_HIP(
        hipMemcpyAsync(s->d_morton, k0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
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
  }
  s->builder = clustered ? MRS_BVH_PLOC : MRS_BVH_LBVH;
  if (n >= 2) rc = collapse4(s, st, leaf_max, scratch, o_q0, o_q1, o_qc, o_is4, o_idx, o_sp4);
  // The scratch must outlive the kernels: wait, then free.
  MRS_TRY_HIP(hipStreamSynchronize(st));
  MRS_TRY_HIP(hipFree(scratch));
  if (rc != MRS_OK) return rc;
  s->root = n >= 2 ? 0u : LEAF_BIT;
  if (n < 2) {
    s->root4 = leaf4_ref(0, 1);
    s->count4 = 0;
  }
  s->bvh_built = true;
  return MRS_OK;
}

}  // namespace mrs
