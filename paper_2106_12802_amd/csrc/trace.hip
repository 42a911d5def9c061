// Wavefront path tracer (Laine, Karras & Aila, "Megakernels considered
// harmful", HPG 2013) for gfx950.
//
// A chunk of paths -- contiguous (sample, pixel) pairs -- is advanced one
// bounce at a time by separate kernels:
//   generate   camera rays (the path state starts at its first shade); skipped
//              when bounce 0 runs the wave traversal, whose kernels compute
//              each camera ray where they need it                 (per path)
//   extend     closest-hit traversal of the BVH4: a wave at a time for the
//              coherent camera rays (scalar node loads, wave-uniform stack),
//              lane by lane for the later bounces (streaming lanes, LDS short
//              stack with a global spill)                     (per live ray)
//   shade      emission, first-hit features, next-event estimation sample,
//              BSDF sample, Russian roulette; appends the surviving rays and
//              the shadow rays to dense queues with one atomic per queue per
//              4-wave block (wave ballot + mbcnt prefix, then an LDS prefix
//              over the block's waves)                          (per live ray)
//   shadow     any-hit traversal; an unoccluded sample adds its contribution
//              to its own path's radiance                       (per shadow ray)
//   tail       the bounces from tail_bounce on, path by path in one launch
//   accumulate per-pixel sums in sample order                   (per pixel)
// Queue sizes stay on the device, so the host enqueues a fixed sequence of
// launches with no read-back.  Each path owns its state slot, and each pixel
// sums its samples in order, so results do not depend on queue order, chunk
// size, grid size or traversal kind.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "mrs_internal.hpp"
#include "devmath.hpp"

namespace mrs {
namespace {

constexpr int TB = 256;        // threads per block of the traversal kernels
constexpr int LDS_STACK = 16;  // stack entries per thread held in LDS
// A BVH4 node pushes at most 3 entries and the collapsed tree is no deeper
// than the binary one; entries beyond MAX_STACK4 are counted as overflows.
constexpr int MAX_STACK4 = 128;
constexpr int MAX_SUB = 4;  // concurrent sub-chunks of a render
constexpr int MAX_BOUNCE_SLOTS = 66;
constexpr float INV_PI = 0.318309886183790671538f;

// Device counter block (uint32 words), reset at the start of every chunk:
constexpr int Q_RAYS = 0;                          // [b] rays entering bounce b
constexpr int Q_SHADOW = MAX_BOUNCE_SLOTS;         // [b] shadow rays made at bounce b
constexpr int Q_FETCH_EXT = 2 * MAX_BOUNCE_SLOTS;  // [b] work fetched by extend at bounce b
constexpr int Q_FETCH_SHD = 3 * MAX_BOUNCE_SLOTS;  // [b] work fetched by shadow at bounce b
constexpr int Q_WORDS = 4 * MAX_BOUNCE_SLOTS;
// stats (uint64): 0 nonfinite, 1 rays, 2 shadow rays, 3 spills, 4 paths, 5 overflow,
// 6/7 extend visits/tests, 8/9 shadow visits/tests

// Rays and shadow rays carry (job << 24 | primitive) in one word.
constexpr uint32_t PRIM24 = 0x00ffffffu;  // "no primitive"
__device__ __forceinline__ uint32_t prim_of(uint32_t w) { return w & PRIM24; }
__device__ __forceinline__ uint32_t job_of(uint32_t w) { return w >> 24; }
__device__ __forceinline__ uint32_t unpack_prim(uint32_t w) {
  const uint32_t p = w & PRIM24;
  return p == PRIM24 ? NO_PRIM : p;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Dense append to two queues for a block of 4 waves: each lane with its
// predicate gets a unique index; one atomic per queue per block (a per-wave
// atomic contends on the one counter chip-wide), and the appended entries of a
// block stay together in the block's order, so a queue keeps the coherence of
// the order its rays were read in.  Must be reached by every thread of the
// block together; the LDS record is free again when it returns.
struct BlockAppend2 {
  uint32_t cnt[4][2];
  uint32_t base[2];
};
__device__ __forceinline__ void block_append2(bool pa, bool pb, uint32_t* ca, uint32_t* cb,
                                              uint32_t& ia, uint32_t& ib, BlockAppend2& sh) {
  const uint64_t ma = __ballot(pa), mb = __ballot(pb);
  const int wave = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    sh.cnt[wave][0] = (uint32_t)__popcll(ma);
    sh.cnt[wave][1] = (uint32_t)__popcll(mb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ta = 0, tb = 0;
    for (int w = 0; w < 4; ++w) {
      const uint32_t a = sh.cnt[w][0], b = sh.cnt[w][1];
      sh.cnt[w][0] = ta;
      sh.cnt[w][1] = tb;
      ta += a;
      tb += b;
    }
    sh.base[0] = ta ? atomicAdd(ca, ta) : 0u;
    sh.base[1] = tb ? atomicAdd(cb, tb) : 0u;
  }
  __syncthreads();
  ia = sh.base[0] + sh.cnt[wave][0] + lanes_below(ma);
  ib = sh.base[1] + sh.cnt[wave][1] + lanes_below(mb);
  __syncthreads();
}

// block_append2 with each entry's place inside its block's segment ordered by
// a small key (0..7; stable within a key): the rays of a wave of the next
// kernel then share one or two keys (a direction octant, a light), which keeps
// their traversals alike.  Same contract as block_append2.
struct BlockAppendKeyed {
  uint32_t cnt[2][8][4];  // queue, key, wave: counts, then exclusive offsets
  uint32_t base[2];
};
__device__ __forceinline__ void block_append2_keyed(bool pa, uint32_t ka, bool pb, uint32_t kb,
                                                    uint32_t* ca, uint32_t* cb, uint32_t& ia,
                                                    uint32_t& ib, BlockAppendKeyed& sh) {
  const int wave = threadIdx.x >> 6;
  uint32_t ra = 0, rb = 0;
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    const uint64_t ma = __ballot(pa && ka == k), mb = __ballot(pb && kb == k);
    if (pa && ka == k) ra = lanes_below(ma);
    if (pb && kb == k) rb = lanes_below(mb);
    if (__lane_id() == 0) {
      sh.cnt[0][k][wave] = (uint32_t)__popcll(ma);
      sh.cnt[1][k][wave] = (uint32_t)__popcll(mb);
    }
  }
  __syncthreads();
  if (wave == 0) {  // lane l: queue l / 32, entry l % 32 = key * 4 + wave, scanned in order
    const int lane = __lane_id(), qq = lane >> 5, i = lane & 31;
    const uint32_t c = sh.cnt[qq][i >> 2][i & 3];
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 32);
      if (i >= d) x += y;
    }
    sh.cnt[qq][i >> 2][i & 3] = x - c;
    if (i == 31) sh.base[qq] = x ? atomicAdd(qq ? cb : ca, x) : 0u;
  }
  __syncthreads();
  ia = pa ? sh.base[0] + sh.cnt[0][ka & 7][wave] + ra : 0u;
  ib = pb ? sh.base[1] + sh.cnt[1][kb & 7][wave] + rb : 0u;
  __syncthreads();
}

__device__ __forceinline__ float safe_rcp(float x) {
  const float ax = fabsf(x) > 1e-20f ? x : copysignf(1e-20f, x);
  return __builtin_amdgcn_rcpf(ax);
}

// Conservative slab test.  The far distance is widened by a few ulp so that
// rounding never culls a box that the ray touches, and a box counts as nearer
// than the best hit so far up to a relative 2^-12: far above the rounding of
// either the box or the triangle distances, so culling never drops a triangle
// that could tie with or beat the best hit, whatever order boxes are visited in.
__device__ __forceinline__ bool slab(float lx, float ly, float lz, float hx, float hy, float hz,
                                     f3 oi, f3 inv, float tbest, float& tnear) {
  const float t0x = fmaf(lx, inv.x, -oi.x), t1x = fmaf(hx, inv.x, -oi.x);
  const float t0y = fmaf(ly, inv.y, -oi.y), t1y = fmaf(hy, inv.y, -oi.y);
  const float t0z = fmaf(lz, inv.z, -oi.z), t1z = fmaf(hz, inv.z, -oi.z);
  const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
  const float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * 1.0000005f;
  tnear = tmin;
  return tmin <= tmax && tmin <= tbest * 1.000244140625f;
}

// The same test on the six plane distances of a box.
__device__ __forceinline__ bool slab_t(float t0x, float t1x, float t0y, float t1y, float t0z,
                                       float t1z, float tbest, float& tnear) {
  const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
  const float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * 1.0000005f;
  tnear = tmin;
  return tmin <= tmax && tmin <= tbest * 1.000244140625f;
}

// Byte c of w as a float (one v_cvt_f32_ubyte).
__device__ __forceinline__ float ubyte(uint32_t w, int c) { return (float)((w >> (8 * c)) & 0xffu); }

struct TraceState {
  float t;
  uint32_t prim;
  float b1, b2;
};

// Traversal arrays as global-address-space pointers: pointers read from the
// job table are generic to the compiler (flat loads); these views give global
// loads.
typedef float vfloat4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const vfloat4 gfloat4;

__device__ __forceinline__ float4 ld4(const gfloat4* p) {
  const vfloat4 v = *p;
  return make_float4(v.x, v.y, v.z, v.w);
}
struct TraceView {
  const gfloat4* nodes;  // BVH4, 8 float4 per node
  const gfloat4* nodes_q;  // the same nodes with quantized child boxes, 4 float4 per node
  const gfloat4* leaf_tri;
  uint32_t root;
  uint32_t nnodes;
  int32_t ntris;
};

// Moller-Trumbore on one triangle given as three float4 (v0 and the primitive
// id, edge 1, edge 2); edges inclusive, t > 0, three excluded primitives.
// any: accept any t < ts.t (shadow rays).  Otherwise accept a closer hit, or an
// equal t with a smaller primitive id.  Both traversals (lane by lane and wave
// by wave) call it, so their hits are bitwise alike.
__device__ __forceinline__ bool isect_tri(const float4 A, const float4 B, const float4 C, f3 o,
                                          f3 d, uint32_t x0, uint32_t x1, uint32_t x2, bool any,
                                          TraceState& ts) {
  const uint32_t prim = __float_as_uint(A.w);
  const f3 e1 = xyz(B), e2 = xyz(C);
  const f3 pv = cross(d, e2);
  const float det = dot(e1, pv);
  const float inv = __builtin_amdgcn_rcpf(det);
  const f3 tv = o - xyz(A);
  const float u = dot(tv, pv) * inv;
  const f3 qv = cross(tv, e1);
  const float v = dot(d, qv) * inv;
  const float t = dot(e2, qv) * inv;
  bool ok = det != 0.0f && u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f && prim != x0 &&
            prim != x1 && prim != x2;
  if (any) {
    ok = ok && t < ts.t;
  } else {
    ok = ok && (t < ts.t || (t == ts.t && prim < ts.prim));
    if (ok) {
      ts.t = t;
      ts.prim = prim;
      ts.b1 = u;
      ts.b2 = v;
    }
  }
  return ok;
}
// The same on triangle `leaf` of the leaf-ordered triangle array.
__device__ __forceinline__ bool isect_leaf(const gfloat4* __restrict__ leaf_tri, uint32_t leaf,
                                           f3 o, f3 d, uint32_t x0, uint32_t x1, uint32_t x2,
                                           bool any, TraceState& ts) {
  const float4 A = ld4(leaf_tri + 3 * leaf), B = ld4(leaf_tri + 3 * leaf + 1),
               C = ld4(leaf_tri + 3 * leaf + 2);
  return isect_tri(A, B, C, o, d, x0, x1, x2, any, ts);
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

struct Stack {
  lds_u32* lds;      // this thread's column: entry k at lds[k * TB]
  uint32_t* spill;   // this thread's global column: entry k at spill[k * stride]
  uint32_t stride;
  int sp;
  uint32_t spills;
  bool overflow;
  __device__ __forceinline__ void push(uint32_t v) {
    if (sp < LDS_STACK) {
      lds[sp * TB] = v;
    } else if (sp < MAX_STACK4) {
      spill[(size_t)(sp - LDS_STACK) * stride] = v;
      ++spills;
    } else {
      overflow = true;
      return;
    }
    ++sp;
  }
  // The LDS read is unconditional (clamped index) and the global read is a
  // branch of its own, so the common case is a plain LDS read rather than one
  // generic load through either address space.
  __device__ __forceinline__ uint32_t pop() {
    --sp;
    const uint32_t top = lds[(sp < LDS_STACK ? sp : LDS_STACK - 1) * TB];
    if (sp < LDS_STACK) return top;
    return spill[(size_t)(sp - LDS_STACK) * stride];
  }
  // Pushes the first `cnt` (0..3) of c, b, a in that order: far to near, so
  // that `a` is popped first.  With room in LDS for three entries (nearly
  // always) the three slots are written unconditionally and sp advances by cnt.
  __device__ __forceinline__ void push_upto3(uint32_t a, uint32_t b, uint32_t c, uint32_t cnt) {
    if (sp + 3 <= LDS_STACK) {
      lds[sp * TB] = cnt == 3 ? c : (cnt == 2 ? b : a);
      lds[(sp + 1) * TB] = cnt == 3 ? b : a;
      lds[(sp + 2) * TB] = a;
      sp += (int)cnt;
      return;
    }
    if (cnt == 3) push(c);
    if (cnt >= 2) push(b);
    if (cnt >= 1) push(a);
  }
};

struct WorkCount {
  uint32_t visits = 0, tests = 0;
  uint32_t ray_steps = 0, max_steps = 0;  // node visits + triangle tests of the current / worst ray
};

__device__ __forceinline__ void cswap(float& ta, uint32_t& ra, float& tb, uint32_t& rb) {
  const bool sw = tb < ta;
  const float t = sw ? tb : ta;
  const uint32_t r = sw ? rb : ra;
  tb = sw ? ta : tb;
  rb = sw ? ra : rb;
  ta = t;
  ra = r;
}

// Per-lane scene view (lanes of a wave may trace different scenes).
__device__ __forceinline__ TraceView lane_view(const SceneView& sv) {
  TraceView t;
  t.nodes = (const gfloat4*)(uintptr_t)sv.nodes;
  t.nodes_q = (const gfloat4*)(uintptr_t)sv.nodes_q;
  t.leaf_tri = (const gfloat4*)(uintptr_t)sv.leaf_tri;
  t.root = sv.root;
  t.nnodes = sv.nnodes;
  t.ntris = sv.ntris;
  return t;
}

// One ray as handed to the traversal.
struct RayIn {
  TraceView sc;
  uint32_t job;  // the ray's job (its scene is the job's)
  f3 o, d;
  uint32_t x0, x1, x2;  // excluded primitives
  float tmax;           // shadow rays: distance to the light point; else infinity
  bool any;             // any hit (shadow ray) rather than the closest hit
};

enum TraceMode { CLOSEST = 0, ANY_HIT = 1, PER_RAY = 2 };

// Streaming four-wide BVH traversal.  Each lane walks its own sequence of
// queue entries first, first + stride, ... < n and starts its next ray as soon
// as the current one is finished, so lanes do not wait for the slowest ray of
// their wave.  Within a ray: the speculative "while-while" loop of Aila &
// Laine (HPG 2009) -- a lane that reaches a leaf parks it and keeps descending
// until every active lane of the wave has a leaf, then the wave intersects the
// parked leaves together.  A ray's visiting order thus depends on the rays
// sharing its wave; the result does not, because box culling is conservative
// (see slab).  Children are visited nearest first (sorting network on the
// entry distances); shadow rays stop at the first occluder.  MODE fixes the
// ray kind (CLOSEST, ANY_HIT) or takes it from each ray (PER_RAY).  IO supplies
// load(qi, RayIn&) and store(qi, const TraceState&, bool occluded, RayIn& next)
// -> bool: true when the lane goes on with `next` for the same queue entry
// (the next segment of a path), false to move to its next entry.  COUNT adds
// node visits and triangle tests to wc (a separate instantiation).
template <int MODE, bool COUNT, bool Q, class IO>
__device__ void trace_stream(IO& io, uint32_t first, uint32_t stride, uint32_t n, Stack& st,
                             WorkCount& wc) {
  uint32_t qi = first;
  bool live = qi < n;
  RayIn r;
  TraceState ts;
  f3 inv, oi;
  uint32_t node = EMPTY4, leaf = EMPTY4;  // next reference to visit; parked leaf
  int32_t budget = 0;
  bool occluded = false;
  auto begin = [&]() {
    ts = TraceState{r.tmax, NO_PRIM, 0.0f, 0.0f};
    inv = F3(safe_rcp(r.d.x), safe_rcp(r.d.y), safe_rcp(r.d.z));
    oi = mul(r.o, inv);
    st.sp = 0;
    occluded = false;
    // every node and leaf is visited at most once per ray in a well-formed tree
    budget = (int32_t)r.sc.nnodes + r.sc.ntris + 2;
    node = leaf = EMPTY4;
    if (r.sc.ntris > 0) {
      if (r.sc.root & LEAF_BIT) leaf = r.sc.root;
      else node = r.sc.root;
    }
  };
  if (live) {
    io.load(qi, r);
    begin();
  }
  while (live) {
    const bool any = MODE == PER_RAY ? r.any : MODE == ANY_HIT;
    // ---- internal nodes (EMPTY4 has the leaf bit set)
    while (!(node & LEAF_BIT) && --budget > 0) {
      if (node >= r.sc.nnodes) {  // keeps a corrupt reference harmless
        node = st.sp ? st.pop() : EMPTY4;
        continue;
      }
      if (COUNT) {
        ++wc.visits;
        ++wc.ray_steps;
      }
      float t0, t1, t2, t3;
      uint32_t r0, r1, r2, r3;
      bool h0, h1, h2, h3;
      // branch-free: every slab test is evaluated, misses become (INFINITY, EMPTY4)
      if (Q) {  // quantized node: plane distance fma(q, 2^e inv, p inv - o inv)
        const gfloat4* nd = r.sc.nodes_q + 4 * node;
        const float4 hd = ld4(nd), qa = ld4(nd + 1), qb = ld4(nd + 2), rf = ld4(nd + 3);
        const uint32_t ex = __float_as_uint(hd.w);
        const float ax = __uint_as_float((ex & 0xffu) << 23) * inv.x;
        const float ay = __uint_as_float(((ex >> 8) & 0xffu) << 23) * inv.y;
        const float az = __uint_as_float(((ex >> 16) & 0xffu) << 23) * inv.z;
        const float bx = fmaf(hd.x, inv.x, -oi.x), by = fmaf(hd.y, inv.y, -oi.y),
                    bz = fmaf(hd.z, inv.z, -oi.z);
        const uint32_t lxw = __float_as_uint(qa.x), lyw = __float_as_uint(qa.y),
                       lzw = __float_as_uint(qa.z), hxw = __float_as_uint(qa.w),
                       hyw = __float_as_uint(qb.x), hzw = __float_as_uint(qb.y);
        r0 = __float_as_uint(rf.x);
        r1 = __float_as_uint(rf.y);
        r2 = __float_as_uint(rf.z);
        r3 = __float_as_uint(rf.w);
#define MRS_QSLAB(c, tc)                                                                    \
  slab_t(fmaf(ubyte(lxw, c), ax, bx), fmaf(ubyte(hxw, c), ax, bx), fmaf(ubyte(lyw, c), ay, by), \
         fmaf(ubyte(hyw, c), ay, by), fmaf(ubyte(lzw, c), az, bz), fmaf(ubyte(hzw, c), az, bz), \
         ts.t, tc)
        h0 = MRS_QSLAB(0, t0) & (r0 != EMPTY4);
        h1 = MRS_QSLAB(1, t1) & (r1 != EMPTY4);
        h2 = MRS_QSLAB(2, t2) & (r2 != EMPTY4);
        h3 = MRS_QSLAB(3, t3) & (r3 != EMPTY4);
#undef MRS_QSLAB
      } else {
        const gfloat4* nd = r.sc.nodes + 8 * node;
        const float4 lx = ld4(nd), ly = ld4(nd + 1), lz = ld4(nd + 2);
        const float4 hx = ld4(nd + 3), hy = ld4(nd + 4), hz = ld4(nd + 5);
        const float4 rf = ld4(nd + 6);
        r0 = __float_as_uint(rf.x);
        r1 = __float_as_uint(rf.y);
        r2 = __float_as_uint(rf.z);
        r3 = __float_as_uint(rf.w);
        h0 = slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, oi, inv, ts.t, t0) & (r0 != EMPTY4);
        h1 = slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, oi, inv, ts.t, t1) & (r1 != EMPTY4);
        h2 = slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, oi, inv, ts.t, t2) & (r2 != EMPTY4);
        h3 = slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, oi, inv, ts.t, t3) & (r3 != EMPTY4);
      }
      t0 = h0 ? t0 : INFINITY;
      t1 = h1 ? t1 : INFINITY;
      t2 = h2 ? t2 : INFINITY;
      t3 = h3 ? t3 : INFINITY;
      r0 = h0 ? r0 : EMPTY4;
      r1 = h1 ? r1 : EMPTY4;
      r2 = h2 ? r2 : EMPTY4;
      r3 = h3 ? r3 : EMPTY4;
      const uint32_t nhit = (uint32_t)h0 + (uint32_t)h1 + (uint32_t)h2 + (uint32_t)h3;
      // sorting network: hits nearest first, misses (INFINITY) last
      cswap(t0, r0, t1, r1);
      cswap(t2, r2, t3, r3);
      cswap(t0, r0, t2, r2);
      cswap(t1, r1, t3, r3);
      cswap(t1, r1, t2, r2);
      // go to the nearest hit child, push the others far to near
      st.push_upto3(r1, r2, r3, nhit > 0 ? nhit - 1 : 0);
      node = nhit > 0 ? r0 : (st.sp ? st.pop() : EMPTY4);
      if ((node & LEAF_BIT) && node != EMPTY4 && leaf == EMPTY4) {
        leaf = node;
        node = st.sp ? st.pop() : EMPTY4;
      }
      if (__all(leaf != EMPTY4)) break;
    }
    // ---- the parked leaf, then leaves that follow on the stack
    while (leaf != EMPTY4 && --budget > 0) {
      const uint32_t f = leaf & 0x00ffffffu, cnt = ((leaf >> 24) & 3u) + 1u;
      if (f + cnt <= (uint32_t)r.sc.ntris) {  // keeps a corrupt reference harmless
        for (uint32_t k = 0; k < cnt; ++k) {
          if (COUNT) {
            ++wc.tests;
            ++wc.ray_steps;
          }
          if (isect_leaf(r.sc.leaf_tri, f + k, r.o, r.d, r.x0, r.x1, r.x2, any, ts) && any) {
            occluded = true;
            break;
          }
        }
      }
      leaf = EMPTY4;
      if (occluded) {
        node = EMPTY4;
        break;
      }
      if ((node & LEAF_BIT) && node != EMPTY4) {
        leaf = node;
        node = st.sp ? st.pop() : EMPTY4;
      }
    }
    if ((node == EMPTY4 && leaf == EMPTY4) || budget <= 0) {  // ray finished
      if (COUNT) {
        wc.max_steps = max(wc.max_steps, wc.ray_steps);
        wc.ray_steps = 0;
      }
      if (io.store(qi, ts, occluded, r)) {
        begin();
      } else {
        qi += stride;
        live = qi < n;
        if (live) {
          io.load(qi, r);
          begin();
        }
      }
    }
  }
}


// ------------------------------------------------------------ wave traversal

// Coherent rays (camera rays: the 64 paths of a wave start in one pixel at 64
// spp, in 16 neighbouring pixels at 4 spp; their shadow rays) are traced a wave
// at a time: the wave walks one tree order together, each lane testing its own
// ray against every node some lane of the wave still needs (Wald et al.,
// "Interactive rendering with coherent ray tracing", 2001, on 64-wide SIMD).
// The node and triangle loads, the stack and the child order are wave-uniform:
// nodes come through the scalar data cache, the stack lives in VGPR lanes, and
// no lane waits on another lane's branch.  A stack entry carries the lanes that
// entered the node's box.  Culling stays per lane and conservative (slab), and
// the triangle test is isect_tri, so each lane's hit is bitwise the one the
// lane-by-lane traversal finds.

typedef __attribute__((address_space(4))) const vfloat4 kfloat4;

// A wave-uniform float4 through the scalar data cache (the address must be
// uniform: it is built from readlane / scalar-load values only).
__device__ __forceinline__ float4 sld4(const kfloat4* p) {
  const vfloat4 v = *p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t rdlane(uint32_t v, uint32_t lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, uint32_t lane) {
  return ((uint64_t)rdlane((uint32_t)(v >> 32), lane) << 32) | rdlane((uint32_t)v, lane);
}

constexpr uint32_t WAVE_STACK = 128;  // entries; as MAX_STACK4 for one lane

// The stack of a wave: entry k = (reference, lane mask) in lane k % 64 of the
// register set k / 64.  sp is wave-uniform.
struct WaveStack {
  uint32_t ref0, lo0, hi0, ref1, lo1, hi1;
  uint32_t sp;
  bool overflow;
  // branch-free over the two register sets (a branch per set makes the
  // compiler keep them in scratch memory)
  __device__ __forceinline__ void push(uint32_t r, uint64_t m) {
    if (sp >= WAVE_STACK) {
      overflow = true;
      return;
    }
    const bool me = __lane_id() == (sp & 63u), s0 = me && sp < 64, s1 = me && sp >= 64;
    const uint32_t mlo = (uint32_t)m, mhi = (uint32_t)(m >> 32);
    ref0 = s0 ? r : ref0;
    lo0 = s0 ? mlo : lo0;
    hi0 = s0 ? mhi : hi0;
    ref1 = s1 ? r : ref1;
    lo1 = s1 ? mlo : lo1;
    hi1 = s1 ? mhi : hi1;
    ++sp;
  }
  __device__ __forceinline__ void pop(uint32_t& r, uint64_t& m) {
    --sp;
    const uint32_t l = sp & 63u;
    const bool first = sp < 64;
    const uint32_t ra = rdlane(ref0, l), rb = rdlane(ref1, l);
    const uint32_t la = rdlane(lo0, l), lb = rdlane(lo1, l);
    const uint32_t ha = rdlane(hi0, l), hb = rdlane(hi1, l);
    r = first ? ra : rb;
    m = ((uint64_t)(first ? ha : hb) << 32) | (first ? la : lb);
  }
};

// Orders two children (entry key, reference, lane mask) by key.
__device__ __forceinline__ void wswap(uint32_t& ka, uint32_t& ra, uint64_t& ma, uint32_t& kb,
                                      uint32_t& rb, uint64_t& mb) {
  if (kb < ka) {
    const uint32_t k = ka, r = ra;
    const uint64_t m = ma;
    ka = kb;
    ra = rb;
    ma = mb;
    kb = k;
    rb = r;
    mb = m;
  }
}

// The lanes `grp` (rays of one scene) walk the tree of `sc` together.  Children
// are entered nearest first as seen by the first lane that enters any of them;
// a child no lane enters is skipped.  ANY: a lane stops at its first occluder,
// and the walk ends when every lane of grp has one.  Visits are bounded by the
// node and triangle counts (each node is entered at most once per walk).
template <bool ANY>
__device__ __forceinline__ void wave_walk(const TraceView& sc, uint64_t grp, const RayIn& r,
                                          f3 inv, f3 oi, TraceState& ts, bool& occluded,
                                          WaveStack& ws) {
  const uint32_t lane = __lane_id();
  const kfloat4* nodes = (const kfloat4*)(uintptr_t)sc.nodes;
  const kfloat4* tris = (const kfloat4*)(uintptr_t)sc.leaf_tri;
  uint32_t node = sc.root;
  uint64_t m = grp, done = 0;
  int32_t budget = (int32_t)sc.nnodes + sc.ntris + 2;
  ws.sp = 0;
  while (--budget > 0) {
    if (!(node & LEAF_BIT)) {
      if (node < sc.nnodes) {
        const bool act = ((m >> lane) & 1ull) != 0;
        const kfloat4* nd = nodes + 8 * node;
        const float4 lx = sld4(nd), ly = sld4(nd + 1), lz = sld4(nd + 2);
        const float4 hx = sld4(nd + 3), hy = sld4(nd + 4), hz = sld4(nd + 5);
        const float4 rf = sld4(nd + 6);
        uint32_t r0 = __float_as_uint(rf.x), r1 = __float_as_uint(rf.y),
                 r2 = __float_as_uint(rf.z), r3 = __float_as_uint(rf.w);
        float t0, t1, t2, t3;
        const bool h0 = act & (r0 != EMPTY4) &
                        slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, oi, inv, ts.t, t0);
        const bool h1 = act & (r1 != EMPTY4) &
                        slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, oi, inv, ts.t, t1);
        const bool h2 = act & (r2 != EMPTY4) &
                        slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, oi, inv, ts.t, t2);
        const bool h3 = act & (r3 != EMPTY4) &
                        slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, oi, inv, ts.t, t3);
        uint64_t m0 = __ballot(h0), m1 = __ballot(h1), m2 = __ballot(h2), m3 = __ballot(h3);
        const uint64_t any_m = m0 | m1 | m2 | m3;
        if (any_m) {
          // keys: the entry distance of the first entering lane (its non-negative
          // float bits order like the floats); children it misses after the rest
          const uint32_t rl = (uint32_t)__builtin_ctzll(any_m);
          const uint32_t FAR = 0x7f800000u, NONE = 0xffffffffu;
          uint32_t k0 = m0 ? rdlane(h0 ? __float_as_uint(t0) & 0x7fffffffu : FAR, rl) : NONE;
          uint32_t k1 = m1 ? rdlane(h1 ? __float_as_uint(t1) & 0x7fffffffu : FAR, rl) : NONE;
          uint32_t k2 = m2 ? rdlane(h2 ? __float_as_uint(t2) & 0x7fffffffu : FAR, rl) : NONE;
          uint32_t k3 = m3 ? rdlane(h3 ? __float_as_uint(t3) & 0x7fffffffu : FAR, rl) : NONE;
          wswap(k0, r0, m0, k1, r1, m1);
          wswap(k2, r2, m2, k3, r3, m3);
          wswap(k0, r0, m0, k2, r2, m2);
          wswap(k1, r1, m1, k3, r3, m3);
          wswap(k1, r1, m1, k2, r2, m2);
          // entered children first (keys below NONE), far ones pushed first
          if (m3) ws.push(r3, m3);
          if (m2) ws.push(r2, m2);
          if (m1) ws.push(r1, m1);
          node = r0;
          m = m0;
          continue;
        }
      }
    } else {
      const uint32_t f = node & 0x00ffffffu, cnt = ((node >> 24) & 3u) + 1u;
      if (f + cnt <= (uint32_t)sc.ntris) {  // keeps a corrupt reference harmless
        const bool act = ((m >> lane) & 1ull) != 0;
        for (uint32_t k = 0; k < cnt; ++k) {
          const kfloat4* tp = tris + 3 * (f + k);
          const float4 A = sld4(tp), B = sld4(tp + 1), C = sld4(tp + 2);
          if (act && !occluded) {
            if (isect_tri(A, B, C, r.o, r.d, r.x0, r.x1, r.x2, ANY, ts) && ANY) occluded = true;
          }
        }
        if (ANY) {
          done |= __ballot(occluded);
          if (!(grp & ~done)) break;
        }
      }
    }
    // next entry with a lane left in it
    bool more = false;
    while (ws.sp) {
      ws.pop(node, m);
      if (ANY) m &= ~done;
      if (m) {
        more = true;
        break;
      }
    }
    if (!more) break;
  }
}

// The 64 queue entries base .. base + 63 (below n) as one wave: each lane
// loads its ray, the lanes of each scene walk its tree together, and each lane
// stores its result.  IO as for trace_stream (store's continuation is not used).
template <bool ANY, class IO>
__device__ __forceinline__ void trace_wave(IO& io, uint32_t base, uint32_t n, WaveStack& ws) {
  const uint32_t qi = base + __lane_id();
  const bool live = qi < n;
  RayIn r{};
  TraceState ts{INFINITY, NO_PRIM, 0.0f, 0.0f};
  f3 inv = F3(1.0f, 1.0f, 1.0f), oi = F3(0.0f, 0.0f, 0.0f);
  bool occluded = false;
  if (live) {
    io.load(qi, r);
    ts.t = r.tmax;
    inv = F3(safe_rcp(r.d.x), safe_rcp(r.d.y), safe_rcp(r.d.z));
    oi = mul(r.o, inv);
  }
  uint64_t todo = __ballot(live);
  while (todo) {
    // the lanes of the first lane's job (lanes of a wave may trace different
    // scenes); the scene is read from the job table with wave-uniform loads
    const uint32_t j0 = rdlane(r.job, (uint32_t)__builtin_ctzll(todo));
    const uint64_t grp = __ballot(live && r.job == j0) & todo;
    todo &= ~grp;
    const SceneView& sv = io.jobs[j0].sv;
    TraceView sc;
    sc.nodes = (const gfloat4*)(uintptr_t)sv.nodes;
    sc.nodes_q = nullptr;
    sc.leaf_tri = (const gfloat4*)(uintptr_t)sv.leaf_tri;
    sc.root = sv.root;
    sc.nnodes = sv.nnodes;
    sc.ntris = sv.ntris;
    if (sc.ntris > 0) wave_walk<ANY>(sc, grp, r, inv, oi, ts, occluded, ws);
  }
  RayIn next;
  if (live) (void)io.store(qi, ts, occluded, next);
}

// ------------------------------------------------------------------ jobs

// Global path index g of a batch: jobs are concatenated, each pixel-major
// (g = first + q * spp + s, q the pixel's place in the tile order below, s
// its sample).
__device__ __forceinline__ uint32_t find_job(const DevJob* __restrict__ jobs, int njobs,
                                             int64_t g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first <= g) lo = mid;
    else hi = mid - 1;
  }
  return (uint32_t)lo;
}

__device__ __forceinline__ uint32_t find_job_pix(const DevJob* __restrict__ jobs, int njobs,
                                                 int64_t i) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].pix_first <= i) lo = mid;
    else hi = mid - 1;
  }
  return (uint32_t)lo;
}

// Pixels are ordered in 8 x 8 tiles (tiles left to right within a tile row,
// pixels row-major inside a tile; edge tiles are cut to the window) and each
// pixel's samples are consecutive, so that the 64 paths of a wave start in a
// few neighbouring pixels (one pixel at 64 spp and more, 16 at 4 spp): their
// camera rays, first hits and shadow rays are coherent.  The full tile rows
// follow a stride permutation (row position p holds tile row p * row_mul mod
// rows_full, row_mul coprime with rows_full and near 0.38 rows_full; a cut
// last row stays last), so that any contiguous range of paths -- a sub-chunk
// traced on its own stream -- samples the whole image and costs about the
// same as any other (the sky at the top of an image is cheap, the ground is
// not).
constexpr uint32_t PT = 8;

// Window pixel (wx, wy) of path-order index q of job J's window.
__device__ __forceinline__ void tile_pixel(const DevJob& J, uint32_t q, uint32_t& wx,
                                           uint32_t& wy) {
  const uint32_t ww = (uint32_t)J.ww, wh = (uint32_t)J.wh;
  const uint32_t rp = q / (PT * ww);
  const uint32_t q0 = q - rp * PT * ww;
  const uint32_t tr = rp < J.rows_full ? rp * J.row_mul % J.rows_full : rp;
  const uint32_t hh = min(PT, wh - PT * tr);
  const uint32_t tc = q0 / (hh * PT);
  const uint32_t q1 = q0 - tc * hh * PT;
  const uint32_t cw = min(PT, ww - PT * tc);
  const uint32_t dy = q1 / cw;
  wy = PT * tr + dy;
  wx = PT * tc + (q1 - dy * cw);
}

// full-image pixel index P and sample s of the path at global index g of job J
__device__ __forceinline__ void path_pixel_sample(const DevJob& J, int64_t g, uint32_t& P,
                                                  uint32_t& s) {
  const int64_t l = g - J.first;
  const uint32_t q = (uint32_t)(l / J.spp);
  s = (uint32_t)(l - (int64_t)q * J.spp);
  uint32_t wx, wy;
  tile_pixel(J, q, wx, wy);
  P = ((uint32_t)J.y0 + wy) * (uint32_t)J.W + ((uint32_t)J.x0 + wx);
}

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(64) void k_store_job(DevJob j, DevJob* dst) {
  if (threadIdx.x == 0) *dst = j;
}

struct SeedTable {
  uint32_t n;
  uint32_t lo[MAX_JOBS], hi[MAX_JOBS];
};

__global__ __launch_bounds__(256) void k_set_seeds(DevJob* jobs, SeedTable t) {
  const uint32_t j = threadIdx.x;
  if (j < t.n) {
    jobs[j].seed_lo = t.lo[j];
    jobs[j].seed_hi = t.hi[j];
  }
}

__global__ __launch_bounds__(256) void k_reset(uint32_t* q, uint32_t n) {
  for (int i = threadIdx.x; i < Q_WORDS; i += blockDim.x) q[i] = (i == Q_RAYS) ? n : 0u;
}

// The camera ray of global path g: its job j, origin o and direction d.
// k_generate stores it; the bounce-0 kernels that skip the stored queue
// (wave traversal and shading, when generation is fused into them) call the
// same function, so every path starts from bitwise the same ray.
__device__ __forceinline__ void camera_ray(const DevJob* __restrict__ jobs, int njobs, int64_t g,
                                           uint32_t& j, f3& o, f3& d) {
  j = find_job(jobs, njobs, g);
  const DevJob& J = jobs[j];
  const SceneView& sc = J.sv;
  uint32_t P, s;
  path_pixel_sample(J, g, P, s);
  const uint32_t py = P / (uint32_t)J.W, px = P - py * (uint32_t)J.W;
  const uint4 r = philox4x32_10(make_uint4(P, s, 0u, 0u), J.seed_lo, J.seed_hi);
  const float sx = ((float)px + unit24(r.x)) / (float)J.W;
  const float sy = ((float)py + unit24(r.y)) / (float)J.H;
  const float aspect = (float)J.W / (float)J.H;
  const float cx = (2.0f * sx - 1.0f) * sc.cam_tan_half * aspect;
  const float cy = (1.0f - 2.0f * sy) * sc.cam_tan_half;
  const f3 f = F3(sc.cam_fx, sc.cam_fy, sc.cam_fz), rr = F3(sc.cam_rx, sc.cam_ry, sc.cam_rz),
           vv = F3(sc.cam_vx, sc.cam_vy, sc.cam_vz);
  d = normalize(f + rr * cx + vv * cy);
  o = F3(sc.cam_px, sc.cam_py, sc.cam_pz);
  // camera effects: translation over the shutter (time from its own Philox
  // block), thin lens (lens sample from words 2, 3, aimed at the point where
  // the pinhole ray meets the focal plane)
  if (J.moving) {
    const uint4 rt = philox4x32_10(make_uint4(P, s, 0u, 4u), J.seed_lo, J.seed_hi);
    const float tau = unit24(rt.x);
    o = o + F3(J.motion_x, J.motion_y, J.motion_z) * tau;
  }
  if (J.lens_r > 0.0f) {
    const f3 Fp = o + d * (J.focus / dot(d, f));
    const float rho = J.lens_r * sqrtf(unit24(r.z));
    float sp, cp;
    sincospif(2.0f * unit24(r.w), &sp, &cp);
    o = o + rr * (rho * cp) + vv * (rho * sp);
    d = normalize(Fp - o);
  }
}

__global__ __launch_bounds__(256) void k_generate(const DevJob* __restrict__ jobs, int njobs,
                                                  int64_t g0, uint32_t n,
                                                  float4* __restrict__ rays) {
  const uint32_t slot = blockIdx.x * 256 + threadIdx.x;
  if (slot >= n) return;
  uint32_t j;
  f3 o, d;
  camera_ray(jobs, njobs, g0 + slot, j, o, d);
  rays[2 * slot] = make_float4(o.x, o.y, o.z, __uint_as_float(slot));
  rays[2 * slot + 1] = make_float4(d.x, d.y, d.z, __uint_as_float((j << 24) | PRIM24));
}

// Queue entries of a traversal wave, 64 at a time.  Static schedule: the
// grid strides over the queue (wave w takes entries w*64 + k*grid).  Dynamic:
// each wave pulls its next 64 entries from a device counter (load balance
// across waves of very different ray costs).
struct WaveQueue {
  uint32_t* ctr;
  uint32_t base, step;
  bool dyn;
  __device__ __forceinline__ uint32_t fetch() {
    uint32_t v = 0;
    if (__lane_id() == 0) v = atomicAdd(ctr, 64u);
    return __builtin_amdgcn_readfirstlane(v);
  }
  __device__ __forceinline__ WaveQueue(uint32_t* c, bool d) : ctr(c), dyn(d) {
    step = gridDim.x * TB;
    base = dyn ? fetch() : blockIdx.x * TB + (threadIdx.x & ~63u);
  }
  __device__ __forceinline__ void next() { base = dyn ? fetch() : base + step; }
};

// GEN: bounce 0 with generation fused in -- queue entry qi is path slot qi and
// its camera ray is computed here instead of read from the queue.
template <bool GEN = false>
struct ExtendIO {
  const DevJob* __restrict__ jobs;
  const float4* __restrict__ rays;
  float4* __restrict__ hits;
  int njobs = 0;
  int64_t g0 = 0;
  __device__ __forceinline__ void load(uint32_t qi, RayIn& r) const {
    r.x1 = r.x2 = NO_PRIM;
    r.tmax = INFINITY;
    r.any = false;
    if (GEN) {
      camera_ray(jobs, njobs, g0 + qi, r.job, r.o, r.d);
      r.sc = lane_view(jobs[r.job].sv);
      r.x0 = NO_PRIM;
      return;
    }
    const float4 R0 = rays[2 * qi], R1 = rays[2 * qi + 1];
    const uint32_t tag = __float_as_uint(R1.w);
    r.job = job_of(tag);
    r.sc = lane_view(jobs[r.job].sv);
    r.o = xyz(R0);
    r.d = xyz(R1);
    r.x0 = unpack_prim(tag);
  }
  __device__ __forceinline__ bool store(uint32_t qi, const TraceState& ts, bool, RayIn&) const {
    hits[qi] = make_float4(ts.t, __uint_as_float(ts.prim), ts.b1, ts.b2);
    return false;
  }
};

// SCHED 0, static: lane sequences gtid, gtid + threads, ...  1, dynamic: a wave
// takes 64 consecutive entries per fetch from a device counter.  One
// instantiation per schedule, so that each kernel holds only its own queue code
// (fewer registers for the static one).
template <int MODE, bool COUNT, bool Q, int SCHED, class IO>
__device__ __forceinline__ void trace_queue(IO& io, uint32_t n, uint32_t* fetch, Stack& st,
                                            WorkCount& wc) {
  if (SCHED == 0) {
    trace_stream<MODE, COUNT, Q>(io, blockIdx.x * TB + threadIdx.x, gridDim.x * TB, n, st, wc);
  } else {
    WaveQueue wq(fetch, true);
    for (; wq.base < n; wq.next())
      trace_stream<MODE, COUNT, Q>(io, wq.base + __lane_id(), 64u, min(n, wq.base + 64u), st,
                                   wc);
  }
}

template <bool COUNT, bool Q, int SCHED>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(7))) void k_extend(const DevJob* __restrict__ jobs, int b,
                                               const float4* __restrict__ rays,
                                               uint32_t* __restrict__ q,
                                               float4* __restrict__ hits,
                                               uint32_t* __restrict__ spill,
                                               unsigned long long* __restrict__ stats) {
  __shared__ uint32_t stk[LDS_STACK * TB];
  const uint32_t n = q[Q_RAYS + b];
  const uint32_t gtid = blockIdx.x * TB + threadIdx.x;
  Stack st{(lds_u32*)stk + threadIdx.x, spill + gtid, gridDim.x * TB, 0, 0u, false};
  WorkCount wc;
  ExtendIO<> io{jobs, rays, hits};
  trace_queue<CLOSEST, COUNT, Q, SCHED>(io, n, q + Q_FETCH_EXT + b, st, wc);
  if (st.spills) atomicAdd(stats + 3, (unsigned long long)st.spills);
  if (st.overflow) atomicAdd(stats + 5, 1ull);
  if (COUNT && wc.visits) atomicAdd(stats + 6, (unsigned long long)wc.visits);
  if (COUNT && wc.tests) atomicAdd(stats + 7, (unsigned long long)wc.tests);
  if (COUNT && wc.max_steps) atomicMax(stats + 10, (unsigned long long)wc.max_steps);
}

__device__ __forceinline__ void onb(f3 n, f3& T, f3& B) {
  // Duff et al., "Building an orthonormal basis, revisited" (JCGT 2017); sign(0) = +1.
  const float s = n.z >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (s + n.z);
  const float b = n.x * n.y * a;
  T = F3(1.0f + s * n.x * n.x * a, s * b, -s * n.x);
  B = F3(b, s + n.y * n.y * a, -n.y);
}

__device__ __forceinline__ float ggx_G1(float a2, float c) {
  return 2.0f * c / (c + sqrtf(a2 + (1.0f - a2) * c * c));
}

__device__ __forceinline__ f3 schlick(f3 f0, float c) {
  const float m = 1.0f - c;
  const float m2 = m * m;
  const float m5 = m2 * m2 * m;
  return F3(f0.x + (1.0f - f0.x) * m5, f0.y + (1.0f - f0.y) * m5, f0.z + (1.0f - f0.z) * m5);
}

// GGX BRDF value (Walter et al. 2007).  The denominator of D is written as
// a^2 cos^2 + |n x h|^2, which equals cos^2 (a^2 - 1) + 1 for unit h but keeps
// full FP32 accuracy when h is close to n.
// GGX D(h) for n.h = ch, with 1 - ch^2 taken as |n x h|^2 (no cancellation
// near the peak of a sharp lobe).
__device__ __forceinline__ float ggx_D(float a2, f3 n, f3 h, float ch) {
  const f3 nh = cross(n, h);
  const float den = a2 * ch * ch + dot(nh, nh);
  return a2 / (3.14159265358979323846f * den * den);
}

__device__ __forceinline__ f3 ggx_eval(f3 f0, float alpha, f3 n, f3 wo, f3 wi, float ci,
                                       float co) {
  const f3 h = normalize(wi + wo);
  const float ch = dot(n, h);
  if (ch <= 0.0f) return F3(0.0f, 0.0f, 0.0f);
  const float a2 = alpha * alpha;
  const float D = ggx_D(a2, n, h, ch);
  const float G = ggx_G1(a2, ci) * ggx_G1(a2, co);
  return schlick(f0, dot(wi, h)) * (D * G / (4.0f * ci * co));
}

// Solid-angle density of reflecting wo into wi when h is drawn with density
// D(h)(n.h): D(h)(n.h) / (4 wo.h).
__device__ __forceinline__ float ggx_pdf(float a2, f3 n, f3 wo, f3 wi) {
  const f3 h = normalize(wi + wo);
  const float ch = dot(n, h), oh = dot(wo, h);
  if (ch <= 0.0f || oh <= 0.0f) return 0.0f;
  return ggx_D(a2, n, h, ch) * ch / (4.0f * oh);
}

// Power-heuristic weight (exponent 2) of a strategy with density a against b
// (Veach & Guibas 1995).
__device__ __forceinline__ float power_weight(float a, float b) {
  return a * a / (a * a + b * b);
}


// The shading of one path vertex (estimator steps E5-E11): emission, the first-hit
// features (b = 0), next-event estimation sample, BSDF sample and Russian
// roulette.  Shared by the wavefront shade kernel and the path-tail kernel, so
// both perform the same arithmetic in the same order.
struct Vertex {
  f3 beta, L;    // throughput and radiance after this vertex's emission
  float pdf;     // solid-angle density of the BSDF sample wi (multiple importance sampling)
  bool cont;     // the path continues from x along wi
  bool shad;     // a shadow ray from x along swi, length sr, carries c if unoccluded
  f3 x, wi, swi, c;
  float sr;
  uint32_t li, prim;
  int lobe;      // render layer of this vertex's BSDF: 0 none, 1 Lambert, 2 GGX
};

// pdf_in: the density of the BSDF sample that led here (0 for camera rays).
__device__ __forceinline__ void shade_vertex(const DevJob& J, int64_t g, int b, f3 o, f3 d,
                                             float4 Hh, f3 beta, f3 L, float pdf_in,
                                             float4* aux2, Vertex& v) {
  const SceneView& sc = J.sv;
  const uint32_t prim = __float_as_uint(Hh.y);
  v.cont = false;
  v.shad = false;
  v.pdf = 0.0f;
  v.prim = prim;
  v.li = 0;
  v.lobe = 0;
  v.x = v.wi = v.swi = v.c = F3(0.0f, 0.0f, 0.0f);
  v.sr = 0.0f;
  if (prim == NO_PRIM) {
    L = L + mul(beta, F3(sc.env_r, sc.env_g, sc.env_b));
    if (aux2) {
      aux2[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      aux2[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    v.beta = beta;
    v.L = L;
    return;
  }
  const float t = Hh.x, b1 = Hh.z, b2 = Hh.w;
  const float4 NG = sc.prim_ng[prim];
  const uint32_t info = __float_as_uint(NG.w);
  f3 ng = xyz(NG);
  f3 ns = ng;
  if (info & PRIM_SMOOTH) {
    const f3 n0 = xyz(sc.prim_n[3 * prim]), n1 = xyz(sc.prim_n[3 * prim + 1]),
             n2 = xyz(sc.prim_n[3 * prim + 2]);
    ns = normalize(n0 * (1.0f - b1 - b2) + n1 * b1 + n2 * b2);
  }
  f3 x = o + d * t;
  const f3 wo = neg(d);
  const bool front = dot(ng, wo) > 0.0f;
  if (!front) {
    ng = neg(ng);
    ns = neg(ns);
  }
  // Rays leave from the hit point lifted along the arrival-side geometric
  // normal by 2^-16 * max(1, |x|_inf): far above FP32 rounding of x, so
  // neither this triangle nor its neighbours are hit again by rounding.
  const float lift = ldexpf(fmaxf(1.0f, fmaxf(fabsf(x.x), fmaxf(fabsf(x.y), fabsf(x.z)))), -16);
  x = x + ng * lift;
  v.x = x;
  const DevMaterial m = sc.mats[info & PRIM_MAT_MASK];
  const int kind = (int)m.emis_kind.w;
  const f3 col = xyz(m.color_alpha);
  v.lobe = kind == MRS_LAMBERT ? 1 : (kind == MRS_GGX ? 2 : 0);
  if (aux2) {
    const f3 alb = kind == MRS_EMITTER ? F3(0, 0, 0) : col;
    aux2[0] = make_float4(alb.x, alb.y, alb.z, ns.x);
    aux2[1] = make_float4(ns.y, ns.z, t, 0.0f);
  }
  const f3 em = xyz(m.emis_kind);
  if (front && (em.x != 0.0f || em.y != 0.0f || em.z != 0.0f)) {
    if (!(info & PRIM_LISTED) || b == 0) {
      L = L + mul(beta, em);
    } else if (J.mis) {
      // a listed light reached by a BSDF sample: weighted against the density
      // with which next-event estimation would have chosen this direction
      // (the light is found by its triangle ids; scenes list few lights)
      for (int i = 0; i < sc.nlights; ++i) {
        const DevLight& lt = sc.lights[i];
        if (lt.tri0 == (int32_t)prim || lt.tri1 == (int32_t)prim) {
          const float cl = dot(xyz(lt.normal), wo);
          if (cl > 0.0f) {
            const float pl = t * t / ((float)sc.nlights * lt.normal.w * cl);
            L = L + mul(beta, em) * power_weight(pdf_in, pl);
          }
          break;
        }
      }
    }
  }
  bool alive = b != J.max_depth && kind != MRS_EMITTER && dot(ns, wo) > 0.0f;
  if (alive) {
    uint32_t P, s;
    path_pixel_sample(J, g, P, s);
    const uint4 bl = philox4x32_10(make_uint4(P, s, 1u + 2u * b, 0u), J.seed_lo, J.seed_hi);
    const uint4 bs = philox4x32_10(make_uint4(P, s, 2u + 2u * b, 0u), J.seed_lo, J.seed_hi);
    const float alpha = m.color_alpha.w;
    const float co = dot(ns, wo);
    // next-event estimation: one light chosen uniformly, area sampling
    if (sc.nlights > 0) {
      const uint32_t li = (uint32_t)(((uint64_t)(bl.x >> 8) * (uint64_t)sc.nlights) >> 24);
      const DevLight& lt = sc.lights[li];
      const float u1 = unit24(bl.y), u2 = unit24(bl.z);
      const f3 y = xyz(lt.corner) + xyz(lt.eu) * u1 + xyz(lt.ev) * u2;
      const f3 dv = y - x;
      const float r2 = dot(dv, dv);
      const float r = sqrtf(r2);
      const f3 w = dv * (1.0f / r);
      const float cs = dot(ns, w), cg = dot(ng, w), cl = -dot(xyz(lt.normal), w);
      v.li = li;
      if (cs > 0.0f && cg > 0.0f && cl > 0.0f) {
        const f3 f = kind == MRS_LAMBERT ? col * INV_PI : ggx_eval(col, alpha, ns, wo, w, cs, co);
        const float geo = cs * cl * ((float)sc.nlights * lt.normal.w) / r2;
        v.c = mul(mul(beta, f), xyz(lt.le)) * geo;
        if (J.mis) {
          const float pl = r2 / ((float)sc.nlights * lt.normal.w * cl);
          const float pb = kind == MRS_LAMBERT ? cs * INV_PI : ggx_pdf(alpha * alpha, ns, wo, w);
          v.c = v.c * power_weight(pl, pb);
        }
        v.swi = w;
        v.sr = r;
        v.shad = true;
      }
    }
    // BSDF sample
    f3 T, B, wi;
    onb(ns, T, B);
    const float v1 = unit24(bs.x), v2 = unit24(bs.y);
    float sp, cp;
    sincospif(2.0f * v2, &sp, &cp);
    if (kind == MRS_LAMBERT) {
      const float rr = sqrtf(v1);
      wi = T * (rr * cp) + B * (rr * sp) + ns * sqrtf(1.0f - v1);
      if (dot(ng, wi) <= 0.0f) alive = false;
      beta = mul(beta, col);
      v.pdf = dot(ns, wi) * INV_PI;
    } else {
      const float a2 = alpha * alpha;
      const float den = 1.0f + (a2 - 1.0f) * v1;
      const float cost = sqrtf((1.0f - v1) / den);
      const float sint = sqrtf(a2 * v1 / den);
      const f3 h = T * (sint * cp) + B * (sint * sp) + ns * cost;
      const float oh = dot(wo, h);
      wi = h * (2.0f * oh) - wo;
      const float ci = dot(ns, wi);
      if (ci <= 0.0f || dot(ng, wi) <= 0.0f) {
        alive = false;
      } else {
        const float ch = dot(ns, h);
        const float G = ggx_G1(a2, ci) * ggx_G1(a2, co);
        beta = mul(beta, schlick(col, oh) * (G * oh / (co * ch)));
        v.pdf = ggx_D(a2, ns, h, ch) * ch / (4.0f * oh);
      }
    }
    if (alive && b >= J.rr_start) {
      const float qq = fminf(0.95f, maxc(beta));
      if (!(unit24(bs.z) < qq)) alive = false;
      else beta = beta * (1.0f / qq);
    }
    v.wi = wi;
  }
  v.cont = alive;
  v.beta = beta;
  v.L = L;
}

// GEN: bounce 0 with generation fused in (queue entry qi is path slot qi; its
// camera ray is recomputed rather than read from the queue).
template <bool SORT, bool GEN>
__global__ __launch_bounds__(256) void k_shade(const DevJob* __restrict__ jobs, int njobs,
                                               int64_t g0, int b,
                                               const float4* __restrict__ rays_in,
                                               const float4* __restrict__ hits,
                                               uint32_t* __restrict__ q,
                                               float4* __restrict__ rays_out,
                                               float4* __restrict__ shadow,
                                               float4* __restrict__ beta_buf,
                                               float4* __restrict__ L_buf,
                                               float4* __restrict__ aux_buf,
                                               float4* __restrict__ lay_buf) {
  const uint32_t n = q[Q_RAYS + b];
  uint32_t* cnt_next = q + Q_RAYS + b + 1;
  uint32_t* cnt_shadow = q + Q_SHADOW + b;
  __shared__ BlockAppend2 sh_app;
  __shared__ BlockAppendKeyed sh_key;
  for (uint32_t base = blockIdx.x * 256; base < n; base += gridDim.x * 256) {
    const uint32_t qi = base + threadIdx.x;
    Vertex v;
    v.cont = v.shad = false;
    v.li = 0;
    v.wi = F3(0.0f, 0.0f, 0.0f);
    uint32_t slot = 0, j = 0;
    if (qi < n) {
      f3 o, d;
      if (GEN) {
        slot = qi;
        camera_ray(jobs, njobs, g0 + qi, j, o, d);
      } else {
        const float4 R0 = rays_in[2 * qi], R1 = rays_in[2 * qi + 1];
        slot = __float_as_uint(R0.w);
        j = job_of(__float_as_uint(R1.w));
        o = xyz(R0);
        d = xyz(R1);
      }
      // a path starts with beta = 1, L = 0 and zero features (nothing is stored
      // for it before its first vertex)
      const float4 Bt = b == 0 ? make_float4(1.0f, 1.0f, 1.0f, 0.0f) : beta_buf[slot];
      const f3 L = b == 0 ? F3(0.0f, 0.0f, 0.0f) : xyz(L_buf[slot]);
      // first-hit features only for jobs that output them
      shade_vertex(jobs[j], g0 + slot, b, o, d, hits[qi], xyz(Bt), L, Bt.w,
                   (b == 0 && jobs[j].out_aux) ? aux_buf + 2 * slot : nullptr, v);
      if (v.cont) beta_buf[slot] = make_float4(v.beta.x, v.beta.y, v.beta.z, v.pdf);
      L_buf[slot] = make_float4(v.L.x, v.L.y, v.L.z, 0.0f);
      // render layers: at the first vertex L holds just the emission seen
      // there (next-event estimates arrive later through the shadow rays)
      if (b == 0 && jobs[j].out_layers)
        lay_buf[slot] = make_float4(v.L.x, v.L.y, v.L.z, (float)v.lobe);
    }
    uint32_t ri, si;
    if (SORT)  // continuing rays by direction octant, shadow rays by light
      block_append2_keyed(v.cont, (v.wi.x < 0.0f) | (v.wi.y < 0.0f) << 1 | (v.wi.z < 0.0f) << 2,
                          v.shad, v.li & 7u, cnt_next, cnt_shadow, ri, si, sh_key);
    else
      block_append2(v.cont, v.shad, cnt_next, cnt_shadow, ri, si, sh_app);
    if (v.cont) {
      rays_out[2 * ri] = make_float4(v.x.x, v.x.y, v.x.z, __uint_as_float(slot));
      rays_out[2 * ri + 1] = make_float4(v.wi.x, v.wi.y, v.wi.z, __uint_as_float((j << 24) | v.prim));
    }
    if (v.shad) {
      shadow[3 * si] = make_float4(v.x.x, v.x.y, v.x.z, __uint_as_float(slot | (v.li << 24)));
      shadow[3 * si + 1] = make_float4(v.swi.x, v.swi.y, v.swi.z, v.sr);
      shadow[3 * si + 2] = make_float4(v.c.x, v.c.y, v.c.z, __uint_as_float((j << 24) | v.prim));
    }
  }
}

struct ShadowIO {
  const DevJob* __restrict__ jobs;
  const float4* __restrict__ shadow;
  float4* __restrict__ L_buf;
  __device__ __forceinline__ void load(uint32_t qi, RayIn& r) const {
    const float4 S0 = shadow[3 * qi], S1 = shadow[3 * qi + 1];
    const uint32_t li = __float_as_uint(S0.w) >> 24;
    const uint32_t ptag = __float_as_uint(shadow[3 * qi + 2].w);
    r.job = job_of(ptag);
    const SceneView& sv = jobs[r.job].sv;
    const DevLight& lt = sv.lights[li];
    r.sc = lane_view(sv);
    r.o = xyz(S0);
    r.d = xyz(S1);
    r.x0 = unpack_prim(ptag);
    r.x1 = (uint32_t)lt.tri0;
    r.x2 = (uint32_t)lt.tri1;
    r.tmax = S1.w;
    r.any = true;
  }
  // an unoccluded sample adds its contribution to its own path's radiance
  __device__ __forceinline__ bool store(uint32_t qi, const TraceState&, bool occluded,
                                        RayIn&) const {
    if (occluded) return false;
    const uint32_t slot = __float_as_uint(shadow[3 * qi].w) & 0xffffffu;
    const float4 S2 = shadow[3 * qi + 2];
    float4 Lv = L_buf[slot];
    Lv.x += S2.x;
    Lv.y += S2.y;
    Lv.z += S2.z;
    L_buf[slot] = Lv;
    return false;
  }
};

template <bool COUNT, bool Q, int SCHED>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(7))) void k_shadow(const DevJob* __restrict__ jobs, int b,
                                               const float4* __restrict__ shadow,
                                               uint32_t* __restrict__ q,
                                               float4* __restrict__ L_buf,
                                               uint32_t* __restrict__ spill,
                                               unsigned long long* __restrict__ stats) {
  __shared__ uint32_t stk[LDS_STACK * TB];
  const uint32_t n = q[Q_SHADOW + b];
  const uint32_t gtid = blockIdx.x * TB + threadIdx.x;
  Stack st{(lds_u32*)stk + threadIdx.x, spill + gtid, gridDim.x * TB, 0, 0u, false};
  WorkCount wc;
  ShadowIO io{jobs, shadow, L_buf};
  trace_queue<ANY_HIT, COUNT, Q, SCHED>(io, n, q + Q_FETCH_SHD + b, st, wc);
  if (st.spills) atomicAdd(stats + 3, (unsigned long long)st.spills);
  if (st.overflow) atomicAdd(stats + 5, 1ull);
  if (COUNT && wc.visits) atomicAdd(stats + 8, (unsigned long long)wc.visits);
  if (COUNT && wc.tests) atomicAdd(stats + 9, (unsigned long long)wc.tests);
  if (COUNT && wc.max_steps) atomicMax(stats + 11, (unsigned long long)wc.max_steps);
}

// Closest hits and shadow rays of bounce b with the wave traversal (trace_wave):
// a wave takes 64 consecutive queue entries at a time, grid-stride or (dyn)
// from the device counter.  Same inputs, outputs and results as k_extend and
// k_shadow.
template <bool GEN>
__global__ __launch_bounds__(TB) void k_extend_wave(const DevJob* __restrict__ jobs, int njobs,
                                                    int64_t g0, int b, int dyn,
                                                    const float4* __restrict__ rays,
                                                    uint32_t* __restrict__ q,
                                                    float4* __restrict__ hits,
                                                    unsigned long long* __restrict__ stats) {
  const uint32_t n = q[Q_RAYS + b];
  ExtendIO<GEN> io{jobs, rays, hits, njobs, g0};
  WaveStack ws{};
  for (WaveQueue wq(q + Q_FETCH_EXT + b, dyn != 0); wq.base < n; wq.next())
    trace_wave<false>(io, wq.base, n, ws);
  if (ws.overflow && __lane_id() == 0) atomicAdd(stats + 5, 1ull);
}

__global__ __launch_bounds__(TB) void k_shadow_wave(const DevJob* __restrict__ jobs, int b,
                                                    int dyn, const float4* __restrict__ shadow,
                                                    uint32_t* __restrict__ q,
                                                    float4* __restrict__ L_buf,
                                                    unsigned long long* __restrict__ stats) {
  const uint32_t n = q[Q_SHADOW + b];
  ShadowIO io{jobs, shadow, L_buf};
  WaveStack ws{};
  for (WaveQueue wq(q + Q_FETCH_SHD + b, dyn != 0); wq.base < n; wq.next())
    trace_wave<true>(io, wq.base, n, ws);
  if (ws.overflow && __lane_id() == 0) atomicAdd(stats + 5, 1ull);
}

// Path tail: the paths still alive at bounce b0 are finished here one by one
// (closest hit, shading, shadow ray, next segment, ...) in a single launch, so
// that the last bounces -- few rays, each launch bounded below by its slowest
// ray -- do not cost a launch sequence per bounce.  Each lane streams over the
// queue like the traversal kernels and, when a segment ends, goes on with the
// next segment of the same path.  The arithmetic is the wavefront's
// (shade_vertex; L += c after an unoccluded shadow ray), so results are
// bitwise those of the wavefront.
struct PathIO {
  const DevJob* __restrict__ jobs;
  const float4* __restrict__ rays;
  float4* __restrict__ beta_buf;
  float4* __restrict__ L_buf;
  int64_t g0;
  int b0;
  uint32_t nrays = 0, nshadow = 0;  // segments traced by this lane
  // the lane's path
  uint32_t slot, j;
  int b;
  f3 beta, L, c, o, d;
  float pdf;  // density of the BSDF sample that led to the next vertex
  f3 next_o, next_d;
  uint32_t next_prim;
  bool cont, in_shadow;

  __device__ __forceinline__ void closest(RayIn& r, f3 ro, f3 rd, uint32_t origin) {
    r.job = j;
    r.sc = lane_view(jobs[j].sv);
    r.o = o = ro;
    r.d = d = rd;
    r.x0 = origin;
    r.x1 = r.x2 = NO_PRIM;
    r.tmax = INFINITY;
    r.any = false;
    in_shadow = false;
    ++nrays;
  }
  __device__ __forceinline__ void load(uint32_t qi, RayIn& r) {
    const float4 R0 = rays[2 * qi], R1 = rays[2 * qi + 1];
    const uint32_t tag = __float_as_uint(R1.w);
    slot = __float_as_uint(R0.w);
    j = job_of(tag);
    b = b0;
    const float4 Bt = beta_buf[slot];
    beta = xyz(Bt);
    pdf = Bt.w;
    L = xyz(L_buf[slot]);
    closest(r, xyz(R0), xyz(R1), unpack_prim(tag));
  }
  __device__ __forceinline__ bool store(uint32_t, const TraceState& ts, bool occluded,
                                        RayIn& r) {
    if (!in_shadow) {
      Vertex v;
      shade_vertex(jobs[j], g0 + slot, b, o, d,
                   make_float4(ts.t, __uint_as_float(ts.prim), ts.b1, ts.b2), beta, L, pdf,
                   nullptr, v);
      beta = v.beta;
      pdf = v.pdf;
      L = v.L;
      cont = v.cont;
      next_o = v.x;
      next_d = v.wi;
      next_prim = v.prim;
      if (v.shad) {
        const DevLight& lt = jobs[j].sv.lights[v.li];
        r.job = j;
        r.sc = lane_view(jobs[j].sv);
        r.o = v.x;
        r.d = v.swi;
        r.x0 = v.prim;
        r.x1 = (uint32_t)lt.tri0;
        r.x2 = (uint32_t)lt.tri1;
        r.tmax = v.sr;
        r.any = true;
        c = v.c;
        in_shadow = true;
        ++nshadow;
        return true;
      }
    } else if (!occluded) {
      L.x += c.x;
      L.y += c.y;
      L.z += c.z;
    }
    if (cont) {
      ++b;
      closest(r, next_o, next_d, next_prim);
      return true;
    }
    L_buf[slot] = make_float4(L.x, L.y, L.z, 0.0f);
    return false;
  }
};

template <bool COUNT, bool Q>
__global__ __launch_bounds__(TB) void k_tail(const DevJob* __restrict__ jobs, int64_t g0, int b0,
                                             const float4* __restrict__ rays,
                                             const uint32_t* __restrict__ q,
                                             float4* __restrict__ beta_buf,
                                             float4* __restrict__ L_buf,
                                             uint32_t* __restrict__ spill,
                                             unsigned long long* __restrict__ stats) {
  __shared__ uint32_t stk[LDS_STACK * TB];
  const uint32_t n = q[Q_RAYS + b0];
  const uint32_t gtid = blockIdx.x * TB + threadIdx.x;
  Stack st{(lds_u32*)stk + threadIdx.x, spill + gtid, gridDim.x * TB, 0, 0u, false};
  WorkCount wc;
  PathIO io;
  io.jobs = jobs;
  io.rays = rays;
  io.beta_buf = beta_buf;
  io.L_buf = L_buf;
  io.g0 = g0;
  io.b0 = b0;
  trace_stream<PER_RAY, COUNT, Q>(io, gtid, gridDim.x * TB, n, st, wc);
  if (io.nrays) {
    atomicAdd(stats + 1, (unsigned long long)io.nrays);
    atomicAdd(stats + 12, (unsigned long long)io.nrays);
  }
  if (io.nshadow) {
    atomicAdd(stats + 2, (unsigned long long)io.nshadow);
    atomicAdd(stats + 13, (unsigned long long)io.nshadow);
  }
  if (st.spills) atomicAdd(stats + 3, (unsigned long long)st.spills);
  if (st.overflow) atomicAdd(stats + 5, 1ull);
  if (COUNT && wc.visits) atomicAdd(stats + 14, (unsigned long long)wc.visits);
  if (COUNT && wc.tests) atomicAdd(stats + 15, (unsigned long long)wc.tests);
  if (COUNT && wc.max_steps) atomicMax(stats + 10, (unsigned long long)wc.max_steps);
}

// Per pixel of every job overlapping the chunk [g0, g0 + n): add its samples of
// the chunk (consecutive slots from slot0 + s_lo), in sample order, to the
// pixel's sums (FP32 or FP64 per job).
template <typename T>
__device__ __forceinline__ void accumulate_pixel(const DevJob& J, char* acc_base, uint32_t pl,
                                                 int64_t s_lo, int64_t s_hi, int64_t slot0,
                                                 int64_t npix, const float4* __restrict__ L_buf,
                                                 const float4* __restrict__ aux_buf,
                                                 const float4* __restrict__ lay_buf,
                                                 uint32_t& bad) {
  T* acc = reinterpret_cast<T*>(acc_base + J.acc_off);
  T* a_rgb = acc + 3 * (int64_t)pl;
  T* a_aux = acc + 3 * npix + 7 * (int64_t)pl;
  T* a_sq = acc + 10 * npix + 3 * (int64_t)pl;
  const bool feats = J.out_aux != nullptr;  // features are only traced for jobs that output them
  const bool lays = J.out_layers != nullptr;
  T* a_lay = acc + 13 * npix + 9 * (int64_t)pl;
  T r = a_rgb[0], gg = a_rgb[1], bb = a_rgb[2];
  T sr = a_sq[0], sg = a_sq[1], sb = a_sq[2];
  T a[7];
  for (int c = 0; c < 7; ++c) a[c] = feats ? a_aux[c] : (T)0;
  T ly[9];
  for (int c = 0; c < 9; ++c) ly[c] = lays ? a_lay[c] : (T)0;
  for (int64_t s = s_lo; s <= s_hi; ++s) {
    const int64_t slot = slot0 + s;
    float4 Lv = L_buf[slot];
    float4 E = lays ? lay_buf[slot] : make_float4(0, 0, 0, 0);
    if (!(isfinite(Lv.x) && isfinite(Lv.y) && isfinite(Lv.z))) {
      Lv = make_float4(0, 0, 0, 0);
      E = make_float4(0, 0, 0, E.w);
      ++bad;
    }
    if (lays) {
      // the emission seen at the first vertex, and the rest to that vertex's lobe
      const int lobe = (int)E.w;
      ly[0] += (T)E.x;
      ly[1] += (T)E.y;
      ly[2] += (T)E.z;
      if (lobe == 1) {
        ly[3] += (T)Lv.x - (T)E.x;
        ly[4] += (T)Lv.y - (T)E.y;
        ly[5] += (T)Lv.z - (T)E.z;
      } else if (lobe == 2) {
        ly[6] += (T)Lv.x - (T)E.x;
        ly[7] += (T)Lv.y - (T)E.y;
        ly[8] += (T)Lv.z - (T)E.z;
      }
    }
    r += (T)Lv.x;
    gg += (T)Lv.y;
    bb += (T)Lv.z;
    sr += (T)Lv.x * (T)Lv.x;
    sg += (T)Lv.y * (T)Lv.y;
    sb += (T)Lv.z * (T)Lv.z;
    if (feats) {
      const float4 A0 = aux_buf[2 * slot], A1 = aux_buf[2 * slot + 1];
      a[0] += (T)A0.x; a[1] += (T)A0.y; a[2] += (T)A0.z; a[3] += (T)A0.w;
      a[4] += (T)A1.x; a[5] += (T)A1.y; a[6] += (T)A1.z;
    }
  }
  a_rgb[0] = r; a_rgb[1] = gg; a_rgb[2] = bb;
  a_sq[0] = sr; a_sq[1] = sg; a_sq[2] = sb;
  if (feats)
    for (int c = 0; c < 7; ++c) a_aux[c] = a[c];
  if (lays)
    for (int c = 0; c < 9; ++c) a_lay[c] = ly[c];
}

__global__ __launch_bounds__(256) void k_accumulate(const DevJob* __restrict__ jobs, int njobs,
                                                    int64_t g0, uint32_t n, int64_t pix_lo,
                                                    int64_t pix_hi,
                                                    const float4* __restrict__ L_buf,
                                                    const float4* __restrict__ aux_buf,
                                                    const float4* __restrict__ lay_buf,
                                                    char* __restrict__ acc_base,
                                                    unsigned long long* __restrict__ stats,
                                                    const uint32_t* __restrict__ qc, int nb) {
  // the chunk's ray counts, once (bounces 0 .. nb-1; the path tail counts its own)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long r = 0, s = 0;
    for (int b = 0; b < nb; ++b) {
      r += qc[Q_RAYS + b];
      s += qc[Q_SHADOW + b];
    }
    atomicAdd(stats + 1, r);
    atomicAdd(stats + 2, s);
    atomicAdd(stats + 4, (unsigned long long)n);
  }
  // i runs over pixels in path order (the chunk's pixels are one range of it)
  const int64_t i = pix_lo + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= pix_hi) return;
  const uint32_t j = find_job_pix(jobs, njobs, i);
  const DevJob& J = jobs[j];
  const int64_t npix = (int64_t)J.ww * J.wh;
  const uint32_t q = (uint32_t)(i - J.pix_first);  // path order of the pixel
  uint32_t wx, wy;
  tile_pixel(J, q, wx, wy);
  const uint32_t pl = wy * (uint32_t)J.ww + wx;  // row-major window pixel (outputs)
  // samples s with g = first + q spp + s in [g0, g0 + n)
  const int64_t base = J.first + (int64_t)q * J.spp;
  const int64_t s_lo = g0 > base ? g0 - base : 0;
  const int64_t s_hi = std::min<int64_t>(J.spp - 1, g0 + n - 1 - base);
  if (s_lo > s_hi) return;
  const int64_t slot0 = base - g0;
  uint32_t bad = 0;
  if (J.fp64)
    accumulate_pixel<double>(J, acc_base, pl, s_lo, s_hi, slot0, npix, L_buf, aux_buf, lay_buf,
                             bad);
  else
    accumulate_pixel<float>(J, acc_base, pl, s_lo, s_hi, slot0, npix, L_buf, aux_buf, lay_buf,
                            bad);
  if (bad) atomicAdd(stats + 0, (unsigned long long)bad);
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

template <typename T>
__device__ __forceinline__ void resolve_pixel(const DevJob& J, const char* acc_base, uint32_t pl,
                                              int64_t npix) {
  const T* acc = reinterpret_cast<const T*>(acc_base + J.acc_off);
  const T inv = (T)1 / (T)J.spp;
  for (int c = 0; c < 3; ++c) J.out_rgb[3 * (int64_t)pl + c] = (float)(acc[3 * (int64_t)pl + c] * inv);
  if (J.out_aux)
    for (int c = 0; c < 7; ++c)
      J.out_aux[7 * (int64_t)pl + c] = (float)(acc[3 * npix + 7 * (int64_t)pl + c] * inv);
  if (J.out_sq)
    for (int c = 0; c < 3; ++c)
      J.out_sq[3 * (int64_t)pl + c] = (float)acc[10 * npix + 3 * (int64_t)pl + c];
  if (J.out_layers)
    for (int c = 0; c < 9; ++c)
      J.out_layers[9 * (int64_t)pl + c] = (float)(acc[13 * npix + 9 * (int64_t)pl + c] * inv);
}

__global__ __launch_bounds__(256) void k_resolve(const DevJob* __restrict__ jobs, int njobs,
                                                 int64_t total_pix, const char* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total_pix) return;
  const uint32_t j = find_job_pix(jobs, njobs, i);
  const DevJob& J = jobs[j];
  const int64_t npix = (int64_t)J.ww * J.wh;
  const uint32_t pl = (uint32_t)(i - J.pix_first);
  if (J.fp64) resolve_pixel<double>(J, acc, pl, npix);
  else resolve_pixel<float>(J, acc, pl, npix);
}

struct DebugHitIO {
  SceneView sv;
  const float* __restrict__ o;
  const float* __restrict__ d;
  const int32_t* __restrict__ skip;
  float* __restrict__ t_out;
  int32_t* __restrict__ prim_out;
  float* __restrict__ b_out;
  __device__ __forceinline__ void load(uint32_t i, RayIn& r) const {
    r.sc = lane_view(sv);
    r.o = F3(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
    r.d = F3(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
    r.x0 = skip ? (uint32_t)skip[i] : NO_PRIM;
    r.x1 = r.x2 = NO_PRIM;
    r.tmax = INFINITY;
    r.any = false;
  }
  __device__ __forceinline__ bool store(uint32_t i, const TraceState& ts, bool, RayIn&) const {
    t_out[i] = ts.t;
    prim_out[i] = ts.prim == NO_PRIM ? -1 : (int32_t)ts.prim;
    b_out[2 * i] = ts.b1;
    b_out[2 * i + 1] = ts.b2;
    return false;
  }
};

template <bool Q>
__global__ __launch_bounds__(TB) void k_debug_hit(SceneView sc, int32_t n,
                                                  const float* __restrict__ o,
                                                  const float* __restrict__ d,
                                                  const int32_t* __restrict__ skip,
                                                  float* __restrict__ t_out,
                                                  int32_t* __restrict__ prim_out,
                                                  float* __restrict__ b_out,
                                                  uint32_t* __restrict__ spill) {
  __shared__ uint32_t stk[LDS_STACK * TB];
  const uint32_t gtid = blockIdx.x * TB + threadIdx.x;
  Stack st{(lds_u32*)stk + threadIdx.x, spill + gtid, gridDim.x * TB, 0, 0u, false};
  WorkCount wc;
  DebugHitIO io{sc, o, d, skip, t_out, prim_out, b_out};
  trace_stream<CLOSEST, false, Q>(io, gtid, gridDim.x * TB, (uint32_t)n, st, wc);
}

__global__ __launch_bounds__(256) void k_debug_philox(int32_t n, const uint32_t* __restrict__ ctr,
                                                      const uint32_t* __restrict__ key,
                                                      uint32_t* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  const uint4 r = philox4x32_10(c, key[2 * i], key[2 * i + 1]);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

// ------------------------------------------------------------------ workspace

// Path state of one stream of renders.  Renders enqueued on one stream share a
// workspace in stream order; each stream, and each batch, has its own, so
// renders on different streams can run concurrently.
// One sub-chunk of a super-chunk: its stream and its slice of the workspace.
struct Sub {
  hipStream_t s;
  int64_t lo;
  uint32_t n;
  unsigned gb;
  size_t o;
  float4* rays[2];
  float4 *hits, *shadow, *beta, *L, *aux, *lay;
  uint32_t *spill, *q;
};

// The part of a render left for its end: the last super-chunk's per-pixel sums
// and the resolve into the outputs.
struct Pending {
  bool active = false;
  hipStream_t st = nullptr;
  int used = 0;
  int nwave = 0;
  Sub sub[MAX_SUB];
};

struct Workspace {
  size_t cap_paths = 0;
  int spill_threads = 0;
  size_t acc_bytes = 0;
  float4* rays[2] = {nullptr, nullptr};
  float4* hits = nullptr;
  float4* shadow = nullptr;
  float4* beta = nullptr;
  float4* L = nullptr;
  float4* aux = nullptr;
  float4* lay = nullptr;  // render layers: first-vertex emission and lobe per path
  uint32_t* spill = nullptr;
  uint32_t* q = nullptr;  // MAX_SUB blocks of Q_WORDS counters
  char* acc = nullptr;    // per-job accumulators (single renders)
  DevJob* one = nullptr;  // device copy of the job of a single render
  unsigned long long* stats = nullptr;  // counters the kernels add to (g_stats)
  int nsub = 0;           // sub-chunk join events created
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[MAX_SUB] = {};
  Pending pend;  // a render begun and not yet ended
  // a render fork not yet used (on stream fork_st, which may be the null
  // stream): its zeroing of the sums and its ev_fork stand for those of the
  // next render begun on that stream
  bool forked = false;
  hipStream_t fork_st = nullptr;
};

// How a render's path space is cut: super-chunks of K * Cs paths; the K
// sub-chunks of Cs paths run concurrently on their own streams, each with
// grids of at most blocks_k traversal blocks.
struct Plan {
  int K;
  int64_t Cs;
  int blocks_k;
};

// A shadow ray carries its path slot in the low 24 bits of a word (the light
// index in the high 8), so a sub-chunk holds at most 2^24 path slots; larger
// chunk_paths values take more super-chunks instead.
constexpr int64_t MAX_SUB_PATHS = int64_t(1) << 24;

Plan make_plan(const mrs_tuning& tu, int64_t total) {
  Plan p;
  p.K = std::max(1, std::min<int>(tu.streams, (int)(total / 65536)));
  const int64_t C = std::max<int64_t>(1, std::min<int64_t>(tu.chunk_paths, total));
  p.Cs = std::min(MAX_SUB_PATHS, ((C + p.K - 1) / p.K + 255) & ~(int64_t)255);
  p.blocks_k = std::max(1, (tu.trace_blocks + p.K - 1) / p.K);
  return p;
}

std::mutex g_mu;  // guards the tables below and the tuning
std::map<hipStream_t, Workspace*> g_stream_ws;
// Sub-chunk streams, shared by every workspace and created once: each takes a
// hardware queue of its own (the runtime has few), so concurrent sub-chunks do
// not end up serialised behind one another on a shared queue.
hipStream_t g_sub[MAX_SUB] = {};
int g_nsub = 0;
unsigned long long* g_stats = nullptr;  // device counters shared by every stream
// defaults: the fastest hybrid 720p frame measured with the clustered BVH
mrs_tuning g_tune = {1 << 23, 8192, 0, 3, 3, 3, MRS_BVH_PLOC, 128, 1, 0, 1, 0, 1};
std::atomic<int> g_conv_small{128};  // g_tune.conv_small_tiles, read without the lock
std::atomic<int> g_net_fused{1};      // g_tune.net_fused_blocks, read without the lock
std::atomic<bool> g_count_work{false};

template <typename T>
void hfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void ws_release(Workspace& w) {
  for (auto*& p : w.rays) hfree(p);
  hfree(w.hits);
  hfree(w.shadow);
  hfree(w.beta);
  hfree(w.L);
  hfree(w.aux);
  hfree(w.lay);
  hfree(w.spill);
  hfree(w.q);
  hfree(w.acc);
  hfree(w.one);
  for (int k = 0; k < w.nsub; ++k) (void)hipEventDestroy(w.ev_join[k]);
  if (w.ev_fork) (void)hipEventDestroy(w.ev_fork);
  w.ev_fork = nullptr;
  w.nsub = 0;
  w.cap_paths = 0;
  w.spill_threads = 0;
  w.acc_bytes = 0;
}

mrs_status ensure_stats() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_stats) return MRS_OK;
  MRS_TRY_HIP(hipMalloc(&g_stats, sizeof(unsigned long long) * MRS_NUM_COUNTERS));
  MRS_TRY_HIP(hipMemset(g_stats, 0, sizeof(unsigned long long) * MRS_NUM_COUNTERS));
  return MRS_OK;
}

// Grows w to hold `paths` path slots, `threads` traversal threads and `nsub`
// sub-chunk streams (device allocations happen only here, and only when the
// workspace grows).
mrs_status ws_ensure(Workspace& w, size_t paths, int threads, int nsub) {
  mrs_status rc = ensure_stats();
  if (rc != MRS_OK) return rc;
  w.stats = g_stats;
  if (!w.q) {
    MRS_TRY_HIP(hipMalloc(&w.q, sizeof(uint32_t) * Q_WORDS * MAX_SUB));
    MRS_TRY_HIP(hipMalloc(&w.one, sizeof(DevJob)));
    MRS_TRY_HIP(hipEventCreateWithFlags(&w.ev_fork, hipEventDisableTiming));
  }
  if (nsub > 0) {
    std::lock_guard<std::mutex> lk(g_mu);
    while (g_nsub < nsub) {
      MRS_TRY_HIP(hipStreamCreateWithFlags(&g_sub[g_nsub], hipStreamNonBlocking));
      ++g_nsub;
    }
  }
  while (w.nsub < nsub) {
    MRS_TRY_HIP(hipEventCreateWithFlags(&w.ev_join[w.nsub], hipEventDisableTiming));
    ++w.nsub;
  }
  if (paths > w.cap_paths) {
    for (auto*& p : w.rays) hfree(p);
    hfree(w.hits);
    hfree(w.shadow);
    hfree(w.beta);
    hfree(w.L);
    hfree(w.aux);
    hfree(w.lay);
    w.cap_paths = 0;
    bool ok = hipMalloc(&w.rays[0], 32 * paths) == hipSuccess &&
              hipMalloc(&w.rays[1], 32 * paths) == hipSuccess &&
              hipMalloc(&w.hits, 16 * paths) == hipSuccess &&
              hipMalloc(&w.shadow, 48 * paths) == hipSuccess &&
              hipMalloc(&w.beta, 16 * paths) == hipSuccess &&
              hipMalloc(&w.L, 16 * paths) == hipSuccess &&
              hipMalloc(&w.aux, 32 * paths) == hipSuccess &&
              hipMalloc(&w.lay, 16 * paths) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      return fail(MRS_ERR_OUT_OF_MEMORY, "render: path-state allocation failed");
    }
    w.cap_paths = paths;
  }
  if (threads > w.spill_threads) {
    hfree(w.spill);
    if (hipMalloc(&w.spill, sizeof(uint32_t) * (MAX_STACK4 - LDS_STACK) * (size_t)threads) !=
        hipSuccess) {
      (void)hipGetLastError();
      w.spill_threads = 0;
      return fail(MRS_ERR_OUT_OF_MEMORY, "render: stack spill allocation failed");
    }
    w.spill_threads = threads;
  }
  return MRS_OK;
}

mrs_status ws_ensure_plan(Workspace& w, const Plan& p) {
  return ws_ensure(w, (size_t)p.K * p.Cs, p.K * p.blocks_k * TB, p.K > 1 ? p.K : 0);
}

mrs_status ws_ensure_acc(Workspace& w, size_t bytes) {
  if (bytes > w.acc_bytes) {
    hfree(w.acc);
    if (hipMalloc(&w.acc, bytes) != hipSuccess) {
      (void)hipGetLastError();
      w.acc_bytes = 0;
      return fail(MRS_ERR_OUT_OF_MEMORY, "render: accumulator allocation failed");
    }
    w.acc_bytes = bytes;
  }
  return MRS_OK;
}

Workspace* stream_workspace(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace*& w = g_stream_ws[st];
  if (!w) w = new Workspace();
  return w;
}

mrs_tuning tuning_snapshot() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tune;
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// rgb 3, features 7, squares 3, then the 9 render-layer sums when asked for
size_t acc_bytes_of(int64_t npix, bool fp64, bool layers) {
  return ((size_t)npix * (layers ? 22 : 13) * (fp64 ? 8 : 4) + 255) & ~(size_t)255;
}

// Per-pixel sums of one super-chunk, in sample order: each sub-chunk, in path
// order, on the caller's stream once that sub-chunk is done (its join event).
mrs_status sum_chunk(Workspace& ws, const DevJob* d_jobs, const std::vector<DevJob>& jobs,
                     const Sub* sub, int used, int nwave, char* acc, hipStream_t st) {
  const int nj = (int)jobs.size();
  for (int k = 0; k < used; ++k) {
    const Sub& u = sub[k];
    if (u.s != st) MRS_TRY_HIP(hipStreamWaitEvent(st, ws.ev_join[k], 0));
    // the chunk's pixels in path order: from the pixel of its first path to
    // the pixel of its last
    int jlo = 0, jhi = nj - 1;
    while (jlo < nj - 1 && jobs[jlo + 1].first <= u.lo) ++jlo;
    while (jhi > 0 && jobs[jhi].first >= u.lo + (int64_t)u.n) --jhi;
    const int64_t pix_lo = jobs[jlo].pix_first + (u.lo - jobs[jlo].first) / jobs[jlo].spp;
    const int64_t pix_hi =
        jobs[jhi].pix_first + (u.lo + (int64_t)u.n - 1 - jobs[jhi].first) / jobs[jhi].spp + 1;
    prof_begin(KID_ACCUMULATE, st);
    k_accumulate<<<cdiv((size_t)(pix_hi - pix_lo), 256), 256, 0, st>>>(
        d_jobs, nj, u.lo, u.n, pix_lo, pix_hi, u.L, u.aux, u.lay, acc, ws.stats, u.q, nwave);
    prof_end(KID_ACCUMULATE, st);
  }
  // the next super-chunk (or render) reuses the slices once these sums have read them
  if (used > 0 && sub[0].s != st) MRS_TRY_HIP(hipEventRecord(ws.ev_fork, st));
  return MRS_OK;
}

// The traversal kernels of a queue schedule (mrs_tuning.schedule).
template <bool COUNT, bool Q>
auto extend_kernel(int sched) {
  return sched == 1 ? k_extend<COUNT, Q, 1> : k_extend<COUNT, Q, 0>;
}
template <bool COUNT, bool Q>
auto shadow_kernel(int sched) {
  return sched == 1 ? k_shadow<COUNT, Q, 1> : k_shadow<COUNT, Q, 0>;
}

// The launch sequence of a batch whose job table is on the device: chunks of at
// most chunk_paths paths over the concatenated path space; per chunk, generate
// (unless bounce 0 computes the camera rays itself), then extend / shade /
// shadow per bounce, then accumulate; finally resolve.
// This enqueues everything but the last super-chunk's sums and the resolve,
// which end_batch enqueues (render_batch does both).
mrs_status begin_batch(Workspace& ws, const mrs_tuning& tu, const DevJob* d_jobs,
                       const std::vector<DevJob>& jobs, char* acc, size_t acc_bytes,
                       hipStream_t st) {
  const int nj = (int)jobs.size();
  int64_t total = 0;
  int max_depth = 0;
  for (const DevJob& J : jobs) {
    total += (int64_t)J.spp * J.ww * J.wh;
    max_depth = std::max(max_depth, (int)J.max_depth);
  }
  const Plan P = make_plan(tu, total);
  // wavefront bounces 0 .. nwave-1; the path tail takes bounces nwave .. max_depth
  const int nwave = std::min(tu.tail_bounce, max_depth + 1);
  const int dyn = tu.schedule;
  const bool qn = tu.bvh_quantized != 0;
  const bool count = g_count_work.load();
  // bounce 0 by the wave traversal: camera rays are computed where they are
  // used (wave traversal, shading) and never stored
  const bool gen_fused = !count && tu.wave_extend > 0;
  unsigned long long* stats = ws.stats;
  const size_t spill_k = (size_t)P.blocks_k * TB * (MAX_STACK4 - LDS_STACK);
  const bool forked = ws.forked && ws.fork_st == st;
  ws.forked = false;
  if (!forked) {
    k_zero_words<<<std::min(4096u, cdiv(acc_bytes / 4, 256)), 256, 0, st>>>((uint32_t*)acc,
                                                                            acc_bytes / 4);
    if (P.K > 1) MRS_TRY_HIP(hipEventRecord(ws.ev_fork, st));
  }
  for (int64_t g0 = 0; g0 < total; g0 += P.K * P.Cs) {
    Sub sub[MAX_SUB];
    int used = 0;
    for (int k = 0; k < P.K && g0 + k * P.Cs < total; ++k, ++used) {
      Sub& u = sub[k];
      u.s = P.K > 1 ? g_sub[k] : st;
      u.lo = g0 + k * P.Cs;
      u.n = (uint32_t)std::min<int64_t>(P.Cs, total - u.lo);
      u.gb = std::min<unsigned>(P.blocks_k, cdiv(u.n, TB));
      u.o = (size_t)k * P.Cs;
      u.rays[0] = ws.rays[0] + 2 * u.o;
      u.rays[1] = ws.rays[1] + 2 * u.o;
      u.hits = ws.hits + u.o;
      u.shadow = ws.shadow + 3 * u.o;
      u.beta = ws.beta + u.o;
      u.L = ws.L + u.o;
      u.aux = ws.aux + 2 * u.o;
      u.lay = ws.lay + u.o;
      u.spill = ws.spill + k * spill_k;
      u.q = ws.q + k * Q_WORDS;
    }
    // Launches are enqueued phase by phase across the sub-chunks so that every
    // stream has work queued early.
    for (int k = 0; k < used; ++k) {
      Sub& u = sub[k];
      if (P.K > 1) MRS_TRY_HIP(hipStreamWaitEvent(u.s, ws.ev_fork, 0));
      k_reset<<<1, 256, 0, u.s>>>(u.q, u.n);
      if (!gen_fused) {
        prof_begin(KID_GENERATE, u.s);
        k_generate<<<cdiv(u.n, 256), 256, 0, u.s>>>(d_jobs, nj, u.lo, u.n, u.rays[0]);
        prof_end(KID_GENERATE, u.s);
      }
    }
    for (int b = 0; b < nwave; ++b) {
      for (int k = 0; k < used; ++k) {
        Sub& u = sub[k];
        prof_begin(KID_EXTEND, u.s);
        if (!count && b < tu.wave_extend) {
          auto wext = b == 0 && gen_fused ? k_extend_wave<true> : k_extend_wave<false>;
          wext<<<u.gb, TB, 0, u.s>>>(d_jobs, nj, u.lo, b, dyn, u.rays[b & 1], u.q, u.hits, stats);
        } else {
          auto ext = count ? (qn ? extend_kernel<true, true>(dyn) : extend_kernel<true, false>(dyn))
                           : (qn ? extend_kernel<false, true>(dyn) : extend_kernel<false, false>(dyn));
          ext<<<u.gb, TB, 0, u.s>>>(d_jobs, b, u.rays[b & 1], u.q, u.hits, u.spill, stats);
        }
        prof_end(KID_EXTEND, u.s);
      }
      for (int k = 0; k < used; ++k) {
        Sub& u = sub[k];
        prof_begin(KID_SHADE, u.s);
        const bool gen = b == 0 && gen_fused;
        auto shd = tu.queue_sort ? (gen ? k_shade<true, true> : k_shade<true, false>)
                                 : (gen ? k_shade<false, true> : k_shade<false, false>);
        shd<<<u.gb, 256, 0, u.s>>>(d_jobs, nj, u.lo, b, u.rays[b & 1], u.hits, u.q,
                                   u.rays[(b + 1) & 1], u.shadow, u.beta, u.L, u.aux, u.lay);
        prof_end(KID_SHADE, u.s);
      }
      if (b < max_depth) {
        for (int k = 0; k < used; ++k) {
          Sub& u = sub[k];
          prof_begin(KID_SHADOW, u.s);
          if (!count && b < tu.wave_shadow) {
            k_shadow_wave<<<u.gb, TB, 0, u.s>>>(d_jobs, b, dyn, u.shadow, u.q, u.L, stats);
          } else {
            auto shd = count ? (qn ? shadow_kernel<true, true>(dyn) : shadow_kernel<true, false>(dyn))
                             : (qn ? shadow_kernel<false, true>(dyn) : shadow_kernel<false, false>(dyn));
            shd<<<u.gb, TB, 0, u.s>>>(d_jobs, b, u.shadow, u.q, u.L, u.spill, stats);
          }
          prof_end(KID_SHADOW, u.s);
        }
      }
    }
    if (nwave <= max_depth) {  // the remaining bounces, path by path
      for (int k = 0; k < used; ++k) {
        Sub& u = sub[k];
        prof_begin(KID_TAIL, u.s);
        auto tail = count ? (qn ? k_tail<true, true> : k_tail<true, false>)
                          : (qn ? k_tail<false, true> : k_tail<false, false>);
        tail<<<u.gb, TB, 0, u.s>>>(d_jobs, u.lo, nwave, u.rays[nwave & 1], u.q, u.beta, u.L,
                                   u.spill, stats);
        prof_end(KID_TAIL, u.s);
      }
    }
    // each sub-chunk's end, recorded on its own stream right after its last launch
    if (P.K > 1)
      for (int k = 0; k < used; ++k) MRS_TRY_HIP(hipEventRecord(ws.ev_join[k], sub[k].s));
    if (g0 + P.K * P.Cs < total) {
      MRS_TRY_STATUS(sum_chunk(ws, d_jobs, jobs, sub, used, nwave, acc, st));
    } else {
      ws.pend.active = true;
      ws.pend.st = st;
      ws.pend.used = used;
      ws.pend.nwave = nwave;
      for (int k = 0; k < used; ++k) ws.pend.sub[k] = sub[k];
    }
  }
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

// The last super-chunk's sums and the resolve into the outputs, on the stream
// the render began on.
mrs_status end_batch(Workspace& ws, const DevJob* d_jobs, const std::vector<DevJob>& jobs,
                     char* acc) {
  const hipStream_t st = ws.pend.st;
  int64_t total_pix = 0;
  for (const DevJob& J : jobs) total_pix += (int64_t)J.ww * J.wh;
  ws.pend.active = false;
  MRS_TRY_STATUS(sum_chunk(ws, d_jobs, jobs, ws.pend.sub, ws.pend.used, ws.pend.nwave, acc, st));
  prof_begin(KID_RESOLVE, st);
  k_resolve<<<cdiv((size_t)total_pix, 256), 256, 0, st>>>(d_jobs, (int)jobs.size(), total_pix,
                                                           acc);
  prof_end(KID_RESOLVE, st);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

mrs_status launch_batch(Workspace& ws, const mrs_tuning& tu, const DevJob* d_jobs,
                        const std::vector<DevJob>& jobs, char* acc, size_t acc_bytes,
                        hipStream_t st) {
  if (ws.pend.active)
    return fail(MRS_ERR_INVALID_ARGUMENT, "render: a split render of this workspace is not ended");
  mrs_status rc = begin_batch(ws, tu, d_jobs, jobs, acc, acc_bytes, st);
  if (rc != MRS_OK) {
    ws.pend.active = false;
    return rc;
  }
  return end_batch(ws, d_jobs, jobs, acc);
}

}  // namespace

namespace {
uint32_t gcd_u(uint32_t a, uint32_t b) {
  while (b) {
    const uint32_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
// x with (a x) mod m == 1 (a coprime with m > 1): extended Euclid.
uint32_t inverse_mod(uint32_t a, uint32_t m) {
  int64_t t = 0, nt = 1, r = m, nr = a % m;
  while (nr) {
    const int64_t q = r / nr;
    t -= q * nt;
    std::swap(t, nt);
    r -= q * nr;
    std::swap(r, nr);
  }
  return (uint32_t)(t < 0 ? t + m : t);
}
}  // namespace

DevJob make_job(const mrs_scene* s, const RenderArgs& a) {
  DevJob J;
  std::memset(&J, 0, sizeof J);
  // stride permutation of the full tile rows (see tile_pixel)
  J.rows_full = (uint32_t)a.wh / PT;
  J.row_mul = J.row_inv = 1;
  if (J.rows_full > 2) {
    uint32_t m = (uint32_t)(0.382 * J.rows_full + 0.5);
    while (gcd_u(m, J.rows_full) != 1) ++m;
    J.row_mul = m;
    J.row_inv = inverse_mod(m, J.rows_full);
  }
  J.sv = s->view;
  J.W = a.W;
  J.H = a.H;
  J.x0 = a.x0;
  J.y0 = a.y0;
  J.ww = a.ww;
  J.wh = a.wh;
  J.spp = a.spp;
  J.max_depth = a.max_depth;
  J.rr_start = a.rr_start;
  J.fp64 = a.fp64 ? 1 : 0;
  J.mis = a.mis ? 1 : 0;
  J.lens_r = a.lens_r;
  J.focus = a.focus;
  J.motion_x = a.motion[0];
  J.motion_y = a.motion[1];
  J.motion_z = a.motion[2];
  J.moving = (a.motion[0] != 0.0f || a.motion[1] != 0.0f || a.motion[2] != 0.0f) ? 1 : 0;
  J.seed_lo = (uint32_t)(a.seed & 0xffffffffu);
  J.seed_hi = (uint32_t)(a.seed >> 32);
  J.out_rgb = a.out_rgb;
  J.out_aux = a.out_aux;
  J.out_sq = a.out_sumsq;
  J.out_layers = a.out_layers;
  return J;
}

mrs_status render(const mrs_scene* s, const RenderArgs& a, hipStream_t st) {
  if (a.max_depth + 2 > MAX_BOUNCE_SLOTS)
    return fail(MRS_ERR_INVALID_ARGUMENT, "render: max_depth too large");
  DevJob J = make_job(s, a);
  J.first = 0;
  J.pix_first = 0;
  J.acc_off = 0;
  const int64_t npix = (int64_t)a.ww * a.wh;
  const mrs_tuning tu = tuning_snapshot();
  Workspace& ws = *stream_workspace(st);
  mrs_status rc = ws_ensure_plan(ws, make_plan(tu, npix * a.spp));
  if (rc != MRS_OK) return rc;
  const size_t ab = acc_bytes_of(npix, a.fp64, a.out_layers != nullptr);
  if ((rc = ws_ensure_acc(ws, ab)) != MRS_OK) return rc;
  k_store_job<<<1, 64, 0, st>>>(J, ws.one);
  std::vector<DevJob> jobs{J};
  return launch_batch(ws, tu, ws.one, jobs, ws.acc, ab, st);
}

// ------------------------------------------------------------ static workspace
// mrs_render_ex_noalloc keeps its whole workspace in one file-scope device
// array: every GPU that loads the library holds its own copy until the process
// ends, and the call allocates nothing.  Capacity: NOALLOC_PATHS resident path
// slots (any spp: more super-chunks), NOALLOC_BLOCKS traversal blocks, and
// NOALLOC_ACC_BYTES of pixel sums (13 FP64 values for each of 2^19 pixels).
constexpr int64_t NOALLOC_PATHS = int64_t(1) << 18;
constexpr int NOALLOC_BLOCKS = 512;
constexpr size_t NOALLOC_ACC_BYTES = size_t(13) * 8 << 19;
constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
// path state per slot: rays 2 x 32 B, hits 16, shadow 48, beta 16, L 16,
// features 32, layers 16
constexpr size_t NA_OFF_RAYS0 = 0;
constexpr size_t NA_OFF_RAYS1 = NA_OFF_RAYS0 + 32 * NOALLOC_PATHS;
constexpr size_t NA_OFF_HITS = NA_OFF_RAYS1 + 32 * NOALLOC_PATHS;
constexpr size_t NA_OFF_SHADOW = NA_OFF_HITS + 16 * NOALLOC_PATHS;
constexpr size_t NA_OFF_BETA = NA_OFF_SHADOW + 48 * NOALLOC_PATHS;
constexpr size_t NA_OFF_L = NA_OFF_BETA + 16 * NOALLOC_PATHS;
constexpr size_t NA_OFF_AUX = NA_OFF_L + 16 * NOALLOC_PATHS;
constexpr size_t NA_OFF_LAY = NA_OFF_AUX + 32 * NOALLOC_PATHS;
constexpr size_t NA_OFF_SPILL = NA_OFF_LAY + 16 * NOALLOC_PATHS;
constexpr size_t NA_OFF_Q =
    NA_OFF_SPILL + al256(sizeof(uint32_t) * (MAX_STACK4 - LDS_STACK) * NOALLOC_BLOCKS * TB);
constexpr size_t NA_OFF_JOB = NA_OFF_Q + al256(sizeof(uint32_t) * Q_WORDS);
constexpr size_t NA_OFF_STATS = NA_OFF_JOB + al256(sizeof(DevJob));
constexpr size_t NA_OFF_ACC = NA_OFF_STATS + al256(sizeof(unsigned long long) * MRS_NUM_COUNTERS);
constexpr size_t NA_BYTES = NA_OFF_ACC + NOALLOC_ACC_BYTES;
static_assert(NA_OFF_RAYS1 % 256 == 0 && NA_OFF_SPILL % 256 == 0 && NA_BYTES % 16 == 0,
              "static workspace layout");

static __device__ __align__(256) uint4 scratch[NA_BYTES / 16];

// Device address of this GPU's copy of `scratch` (host code must never use the
// array's name as an address: it is a host-side stand-in).  Looked up once per
// device, with that device current.
constexpr int NA_MAX_DEVICES = 64;
char* g_scratch_ptr[NA_MAX_DEVICES] = {};

mrs_status scratch_base(char** out) {
  int dev = 0;
  MRS_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAX_DEVICES)
    return fail(MRS_ERR_UNSUPPORTED, "mrs_render_ex_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(MRS_ERR_DEVICE, std::string("mrs_render_ex_noalloc: hipGetSymbolAddress: ") +
                                      hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return MRS_OK;
}

mrs_status render_noalloc(const mrs_scene* s, const RenderArgs& a, hipStream_t st) {
  if (a.max_depth + 2 > MAX_BOUNCE_SLOTS)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_render_ex_noalloc: max_depth too large");
  const int64_t npix = (int64_t)a.ww * a.wh;
  const size_t ab = acc_bytes_of(npix, a.fp64, a.out_layers != nullptr);
  if (ab > NOALLOC_ACC_BYTES)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_render_ex_noalloc: the window needs " + std::to_string(ab) +
                    " bytes of pixel sums; the static workspace holds " +
                    std::to_string(NOALLOC_ACC_BYTES) +
                    " (2^19 pixels with FP64 sums, 2^20 with FP32 sums, fewer with render "
                    "layers): render it in windows");
  char* base = nullptr;
  mrs_status rc = scratch_base(&base);
  if (rc != MRS_OK) return rc;
  mrs_tuning tu = tuning_snapshot();
  tu.streams = 1;  // the caller's stream only: no internal streams or events
  tu.chunk_paths = (int32_t)std::min<int64_t>(tu.chunk_paths, NOALLOC_PATHS);
  tu.trace_blocks = std::min(tu.trace_blocks, NOALLOC_BLOCKS);
  Workspace ws;
  ws.cap_paths = (size_t)NOALLOC_PATHS;
  ws.spill_threads = NOALLOC_BLOCKS * TB;
  ws.rays[0] = reinterpret_cast<float4*>(base + NA_OFF_RAYS0);
  ws.rays[1] = reinterpret_cast<float4*>(base + NA_OFF_RAYS1);
  ws.hits = reinterpret_cast<float4*>(base + NA_OFF_HITS);
  ws.shadow = reinterpret_cast<float4*>(base + NA_OFF_SHADOW);
  ws.beta = reinterpret_cast<float4*>(base + NA_OFF_BETA);
  ws.L = reinterpret_cast<float4*>(base + NA_OFF_L);
  ws.aux = reinterpret_cast<float4*>(base + NA_OFF_AUX);
  ws.lay = reinterpret_cast<float4*>(base + NA_OFF_LAY);
  ws.spill = reinterpret_cast<uint32_t*>(base + NA_OFF_SPILL);
  ws.q = reinterpret_cast<uint32_t*>(base + NA_OFF_Q);
  ws.one = reinterpret_cast<DevJob*>(base + NA_OFF_JOB);
  ws.stats = reinterpret_cast<unsigned long long*>(base + NA_OFF_STATS);
  ws.acc = base + NA_OFF_ACC;
  ws.acc_bytes = NOALLOC_ACC_BYTES;
  const Plan P = make_plan(tu, npix * a.spp);
  if (P.K != 1 || P.Cs > NOALLOC_PATHS || P.blocks_k > NOALLOC_BLOCKS)
    return fail(MRS_ERR_DEVICE, "mrs_render_ex_noalloc: internal plan exceeds the workspace");
  DevJob J = make_job(s, a);
  J.first = 0;
  J.pix_first = 0;
  J.acc_off = 0;
  ProfPause pause;  // kernel timing would create events
  // the counters of this call start at zero and are not added to mrs_get_counters
  k_zero_words<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(ws.stats), 2 * MRS_NUM_COUNTERS);
  k_store_job<<<1, 64, 0, st>>>(J, ws.one);
  std::vector<DevJob> jobs{J};
  return launch_batch(ws, tu, ws.one, jobs, ws.acc, ab, st);
}

}  // namespace mrs

// A batch owns its job table, accumulators and path workspace, sized at
// creation with the tuning current then, so rendering it allocates nothing.
struct mrs_batch {
  std::vector<mrs::DevJob> jobs;
  mrs::DevJob* d_jobs = nullptr;
  char* d_acc = nullptr;
  size_t acc_bytes = 0;
  mrs_tuning tune;
  mrs::Workspace ws;
};

namespace mrs {

void batch_destroy(mrs_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  hfree(b->d_jobs);
  hfree(b->d_acc);
  ws_release(b->ws);
  delete b;
}

mrs_status batch_create(const std::vector<DevJob>& jobs, mrs_batch** out) {
  for (const DevJob& J : jobs)
    if (J.max_depth + 2 > MAX_BOUNCE_SLOTS)
      return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_create: max_depth too large");
  mrs_batch* b = new mrs_batch();
  b->jobs = jobs;
  b->tune = tuning_snapshot();
  int64_t first = 0, pix = 0;
  size_t off = 0;
  for (DevJob& J : b->jobs) {
    const int64_t npix = (int64_t)J.ww * J.wh;
    J.first = first;
    J.pix_first = pix;
    J.acc_off = (int64_t)off;
    first += npix * J.spp;
    pix += npix;
    off += acc_bytes_of(npix, J.fp64 != 0, J.out_layers != nullptr);
  }
  b->acc_bytes = off;
  mrs_status rc = ws_ensure_plan(b->ws, make_plan(b->tune, first));
  if (rc == MRS_OK && (hipMalloc(&b->d_jobs, sizeof(DevJob) * b->jobs.size()) != hipSuccess ||
                       hipMalloc(&b->d_acc, b->acc_bytes) != hipSuccess)) {
    (void)hipGetLastError();
    rc = fail(MRS_ERR_OUT_OF_MEMORY, "mrs_batch_create: device allocation failed");
  }
  if (rc == MRS_OK) {
    hipError_t e = hipMemcpy(b->d_jobs, b->jobs.data(), sizeof(DevJob) * b->jobs.size(),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = check_hip(e, "mrs_batch_create: job table upload");
  }
  if (rc != MRS_OK) {
    batch_destroy(b);
    return rc;
  }
  *out = b;
  return MRS_OK;
}

mrs_status batch_render(mrs_batch* b, hipStream_t st) {
  return launch_batch(b->ws, b->tune, b->d_jobs, b->jobs, b->d_acc, b->acc_bytes, st);
}

mrs_status batch_render_begin(mrs_batch* b, hipStream_t st) {
  if (b->ws.pend.active)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_batch_render_begin: the batch's previous render is not ended");
  mrs_status rc = begin_batch(b->ws, b->tune, b->d_jobs, b->jobs, b->d_acc, b->acc_bytes, st);
  if (rc != MRS_OK) b->ws.pend.active = false;
  return rc;
}

// The first part of begin_batch on its own: clear the sums and record the
// point the sub-chunk streams start from.
mrs_status batch_render_fork(mrs_batch* b, hipStream_t st) {
  if (b->ws.pend.active)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_batch_render_fork: the batch's previous render is not ended");
  int64_t total = 0;
  for (const DevJob& J : b->jobs) total += (int64_t)J.spp * J.ww * J.wh;
  const Plan P = make_plan(b->tune, total);
  k_zero_words<<<std::min(4096u, cdiv(b->acc_bytes / 4, 256)), 256, 0, st>>>(
      (uint32_t*)b->d_acc, b->acc_bytes / 4);
  if (P.K > 1) MRS_TRY_HIP(hipEventRecord(b->ws.ev_fork, st));
  MRS_TRY_HIP(hipGetLastError());
  b->ws.forked = true;
  b->ws.fork_st = st;
  return MRS_OK;
}

mrs_status batch_render_end(mrs_batch* b, hipStream_t st) {
  if (!b->ws.pend.active)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_render_end: no render of the batch begun");
  if (b->ws.pend.st != st)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_batch_render_end: not the stream mrs_batch_render_begin ran on");
  return end_batch(b->ws, b->d_jobs, b->jobs, b->d_acc);
}

mrs_status batch_set_seeds(mrs_batch* b, const uint64_t* seeds, hipStream_t st) {
  // a fork recorded before the new seeds would let the sub-chunk streams start
  // without them: the next render records its own
  b->ws.forked = false;
  SeedTable t;
  std::memset(&t, 0, sizeof t);
  t.n = (uint32_t)b->jobs.size();
  for (uint32_t j = 0; j < t.n; ++j) {
    t.lo[j] = (uint32_t)(seeds[j] & 0xffffffffu);
    t.hi[j] = (uint32_t)(seeds[j] >> 32);
    b->jobs[j].seed_lo = t.lo[j];
    b->jobs[j].seed_hi = t.hi[j];
  }
  k_set_seeds<<<1, 256, 0, st>>>(b->d_jobs, t);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

void release_workspaces() {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_stream_ws) {
    ws_release(*kv.second);
    delete kv.second;
  }
  g_stream_ws.clear();
}

mrs_status debug_closest_hit(const mrs_scene* s, int32_t n, const float* o, const float* d,
                             const int32_t* skip, float* t, int32_t* prim, float* b,
                             hipStream_t st) {
  if (n <= 0) return MRS_OK;
  const unsigned blocks = std::min(cdiv((size_t)n, TB), 1024u);
  Workspace& ws = *stream_workspace(st);
  mrs_status rc = ws_ensure(ws, 1, (int)(blocks * TB), 0);
  if (rc != MRS_OK) return rc;
  if (tuning_snapshot().bvh_quantized)
    k_debug_hit<true><<<blocks, TB, 0, st>>>(s->view, n, o, d, skip, t, prim, b, ws.spill);
  else
    k_debug_hit<false><<<blocks, TB, 0, st>>>(s->view, n, o, d, skip, t, prim, b, ws.spill);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

mrs_status debug_philox(int32_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                        hipStream_t st) {
  if (n <= 0) return MRS_OK;
  k_debug_philox<<<cdiv((size_t)n, 256), 256, 0, st>>>(n, ctr, key, out);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

mrs_status get_counters(int64_t* out, bool reset, hipStream_t st) {
  for (int i = 0; i < MRS_NUM_COUNTERS; ++i) out[i] = 0;
  if (!g_stats) return MRS_OK;
  unsigned long long h[MRS_NUM_COUNTERS];
  MRS_TRY_HIP(hipMemcpyAsync(h, g_stats, sizeof(h), hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < MRS_NUM_COUNTERS; ++i) out[i] = (int64_t)h[i];
  if (reset) {
    k_zero_words<<<1, 256, 0, st>>>((uint32_t*)g_stats, 2 * MRS_NUM_COUNTERS);
    MRS_TRY_HIP(hipGetLastError());
  }
  return MRS_OK;
}

void get_tuning(mrs_tuning* t) { *t = tuning_snapshot(); }

void set_count_work(bool on) { g_count_work = on; }

mrs_status set_tuning(const mrs_tuning* t) {
  if (t->chunk_paths < 256 || t->chunk_paths > (1 << 26))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: chunk_paths must be in [256, 2^26]");
  if (t->trace_blocks < 1 || t->trace_blocks > 65536)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: trace_blocks must be in [1, 65536]");
  if (t->schedule != 0 && t->schedule != 1)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: schedule must be 0 or 1");
  if (t->bvh_leaf_max < 1 || t->bvh_leaf_max > LEAF4_MAX)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: bvh_leaf_max must be in [1, 4]");
  if (t->streams < 1 || t->streams > MAX_SUB)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: streams must be in [1, 4]");
  if (t->tail_bounce < 1 || t->tail_bounce > 65)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: tail_bounce must be in [1, 65]");
  if (t->bvh_builder != MRS_BVH_LBVH && t->bvh_builder != MRS_BVH_PLOC)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: bvh_builder must be 0 or 1");
  if (t->conv_small_tiles < 0 || t->conv_small_tiles > (1 << 30))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: conv_small_tiles must be in [0, 2^30]");
  if (t->queue_sort != 0 && t->queue_sort != 1)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: queue_sort must be 0 or 1");
  if (t->bvh_quantized != 0 && t->bvh_quantized != 1)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: bvh_quantized must be 0 or 1");
  if (t->wave_extend < 0 || t->wave_extend > 65 || t->wave_shadow < 0 || t->wave_shadow > 65)
    return fail(MRS_ERR_INVALID_ARGUMENT,
                "mrs_set_tuning: wave_extend and wave_shadow must be in [0, 65]");
  if (t->net_fused_blocks != 0 && t->net_fused_blocks != 1)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: net_fused_blocks must be 0 or 1");
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune = *t;
  g_conv_small = t->conv_small_tiles;
  g_net_fused = t->net_fused_blocks;
  return MRS_OK;
}

int conv_small_tiles() { return g_conv_small.load(std::memory_order_relaxed); }
int net_fused_blocks() { return g_net_fused.load(std::memory_order_relaxed); }

}  // namespace mrs
