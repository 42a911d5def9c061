// Wavefront path tracer (Laine, Karras & Aila, "Megakernels considered
// harmful", HPG 2013) for gfx950.
//
// A chunk of paths -- contiguous (sample, pixel) pairs -- is advanced one
// bounce at a time by separate kernels:
//   generate   camera rays, path state init                    (per path)
//   extend     closest-hit LBVH traversal, LDS short stack      (per live ray)
//   shade      emission, first-hit features, next-event estimation sample,
//              BSDF sample, Russian roulette; appends the surviving rays and
//              the shadow rays to dense queues with one atomic per wave
//              (ballot + mbcnt prefix)                          (per live ray)
//   shadow     any-hit traversal; an unoccluded sample adds its contribution
//              to its own path's radiance                       (per shadow ray)
//   accumulate per-pixel sums in sample order                   (per pixel)
// Queue sizes stay on the device, so the host enqueues a fixed sequence of
// launches with no read-back.  Each path owns its state slot, and each pixel
// sums its samples in order, so results do not depend on queue order, chunk
// size or grid size.
#include <algorithm>
#include <vector>

#include "mrs_internal.hpp"
#include "devmath.hpp"

namespace mrs {
namespace {

constexpr int TB = 256;        // threads per block of the traversal kernels
constexpr int LDS_STACK = 16;  // stack entries per thread held in LDS
constexpr int MAX_BOUNCE_SLOTS = 66;
constexpr float INV_PI = 0.318309886183790671538f;

// Layout of the device counter block (uint32 words, then uint64 stats).
constexpr int Q_RAYS = 0;                      // [b] rays entering bounce b
constexpr int Q_SHADOW = MAX_BOUNCE_SLOTS;     // [b] shadow rays made at bounce b
constexpr int Q_WORDS = 2 * MAX_BOUNCE_SLOTS;  // uint32 words before the stats
// stats (uint64): 0 nonfinite, 1 rays, 2 shadow rays, 3 spills, 4 paths, 5 overflow

struct ChunkGeom {
  int32_t W, H, x0, y0, ww;
  int32_t s0, np, p0;
  uint32_t seed_lo, seed_hi;
  int32_t max_depth, rr_start;
};

__device__ __forceinline__ void slot_pixel_sample(const ChunkGeom& g, uint32_t slot, uint32_t& P,
                                                  uint32_t& s, uint32_t& pl) {
  const uint32_t k = slot / (uint32_t)g.np;
  pl = (uint32_t)g.p0 + (slot - k * (uint32_t)g.np);
  s = (uint32_t)g.s0 + k;
  const uint32_t wy = pl / (uint32_t)g.ww, wx = pl - wy * (uint32_t)g.ww;
  P = ((uint32_t)g.y0 + wy) * (uint32_t)g.W + ((uint32_t)g.x0 + wx);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Dense append: every lane with `pred` gets a unique index in the queue; one
// atomic per wave.  Must be reached by all lanes of the wave together.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0;
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __builtin_amdgcn_readlane(base, leader);
  return base + lanes_below(m);
}

__device__ __forceinline__ float safe_rcp(float x) {
  const float ax = fabsf(x) > 1e-20f ? x : copysignf(1e-20f, x);
  return __builtin_amdgcn_rcpf(ax);
}

// Conservative slab test; the far distance is widened by a few ulp so that
// rounding never culls a box that the ray touches.
__device__ __forceinline__ bool slab(float lx, float ly, float lz, float hx, float hy, float hz,
                                     f3 oi, f3 inv, float tbest, float& tnear) {
  const float t0x = fmaf(lx, inv.x, -oi.x), t1x = fmaf(hx, inv.x, -oi.x);
  const float t0y = fmaf(ly, inv.y, -oi.y), t1y = fmaf(hy, inv.y, -oi.y);
  const float t0z = fmaf(lz, inv.z, -oi.z), t1z = fmaf(hz, inv.z, -oi.z);
  const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
  const float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * 1.0000005f;
  tnear = tmin;
  return tmin <= tmax && tmin <= tbest;
}

struct TraceState {
  float t;
  uint32_t prim;
  float b1, b2;
};

// Moller-Trumbore against one leaf; edges inclusive, t > 0, three excluded
// primitives.  ANY: accept any t < ts.t (shadow rays).  Otherwise accept a
// closer hit, or an equal t with a smaller primitive id.
template <bool ANY>
__device__ __forceinline__ bool isect_leaf(const float4* __restrict__ leaf_tri, uint32_t leaf,
                                           f3 o, f3 d, uint32_t x0, uint32_t x1, uint32_t x2,
                                           TraceState& ts) {
  const float4 A = leaf_tri[3 * leaf], B = leaf_tri[3 * leaf + 1], C = leaf_tri[3 * leaf + 2];
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
  if (ANY) {
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

struct Stack {
  uint32_t* lds;     // this thread's column: entry k at lds[k * TB]
  uint32_t* spill;   // this thread's global column: entry k at spill[k * stride]
  uint32_t stride;
  int sp;
  uint32_t spills;
  bool overflow;
  __device__ __forceinline__ void push(uint32_t v) {
    if (sp < LDS_STACK) {
      lds[sp * TB] = v;
    } else if (sp < MAX_STACK) {
      spill[(size_t)(sp - LDS_STACK) * stride] = v;
      ++spills;
    } else {
      overflow = true;
      return;
    }
    ++sp;
  }
  __device__ __forceinline__ uint32_t pop() {
    --sp;
    return sp < LDS_STACK ? lds[sp * TB] : spill[(size_t)(sp - LDS_STACK) * stride];
  }
};

struct WorkCount {
  uint32_t visits = 0, tests = 0;
};

// Returns true for ANY when an occluder was found; fills ts otherwise.  COUNT
// adds node visits and triangle tests to wc (a separate instantiation).
template <bool ANY, bool COUNT>
__device__ bool traverse(const SceneView& sc, f3 o, f3 d, uint32_t x0, uint32_t x1, uint32_t x2,
                         Stack& st, TraceState& ts, WorkCount& wc) {
  if (sc.ntris == 0) return false;
  if (sc.root & LEAF_BIT) {
    if (COUNT) ++wc.tests;
    return isect_leaf<ANY>(sc.leaf_tri, 0, o, d, x0, x1, x2, ts);
  }
  const f3 inv = F3(safe_rcp(d.x), safe_rcp(d.y), safe_rcp(d.z));
  const f3 oi = mul(o, inv);
  uint32_t node = 0;
  st.sp = 0;
  const uint32_t ninternal = (uint32_t)sc.ntris - 1u;
  // A well-formed tree visits each internal node at most once per ray.
  for (uint32_t visits = 0; visits < ninternal; ++visits) {
    const float4* nd = sc.nodes + 4 * (size_t)node;
    const float4 a = nd[0], b = nd[1], c = nd[2], r = nd[3];
    if (COUNT) ++wc.visits;
    float tl, tr;
    bool hl = slab(a.x, a.y, a.z, a.w, b.x, b.y, oi, inv, ts.t, tl);
    bool hr = slab(b.z, b.w, c.x, c.y, c.z, c.w, oi, inv, ts.t, tr);
    const uint32_t cl = __float_as_uint(r.x), cr = __float_as_uint(r.y);
    // references always lie inside the tree; the checks keep a corrupt one harmless
    if ((cl & LEAF_BIT) ? (cl & ~LEAF_BIT) >= (uint32_t)sc.ntris : cl >= ninternal) hl = false;
    if ((cr & LEAF_BIT) ? (cr & ~LEAF_BIT) >= (uint32_t)sc.ntris : cr >= ninternal) hr = false;
    if (hl && (cl & LEAF_BIT)) {
      if (COUNT) ++wc.tests;
      if (isect_leaf<ANY>(sc.leaf_tri, cl & ~LEAF_BIT, o, d, x0, x1, x2, ts) && ANY) return true;
      hl = false;
    }
    if (hr && (cr & LEAF_BIT)) {
      if (COUNT) ++wc.tests;
      if (isect_leaf<ANY>(sc.leaf_tri, cr & ~LEAF_BIT, o, d, x0, x1, x2, ts) && ANY) return true;
      hr = false;
    }
    if (hl && hr) {
      const bool lfirst = tl <= tr;
      st.push(lfirst ? cr : cl);
      node = lfirst ? cl : cr;
    } else if (hl) {
      node = cl;
    } else if (hr) {
      node = cr;
    } else {
      if (st.sp == 0) break;
      node = st.pop();
    }
  }
  return false;
}

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(256) void k_reset(uint32_t* q, uint32_t n) {
  for (int i = threadIdx.x; i < Q_WORDS; i += blockDim.x) q[i] = (i == Q_RAYS) ? n : 0u;
}

__global__ __launch_bounds__(256) void k_generate(ChunkGeom g, SceneView sc, uint32_t n,
                                                  float4* __restrict__ rays,
                                                  float4* __restrict__ beta,
                                                  float4* __restrict__ L,
                                                  float4* __restrict__ aux) {
  const uint32_t slot = blockIdx.x * 256 + threadIdx.x;
  if (slot >= n) return;
  uint32_t P, s, pl;
  slot_pixel_sample(g, slot, P, s, pl);
  const uint32_t py = P / (uint32_t)g.W, px = P - py * (uint32_t)g.W;
  const uint4 r = philox4x32_10(make_uint4(P, s, 0u, 0u), g.seed_lo, g.seed_hi);
  const float sx = ((float)px + unit24(r.x)) / (float)g.W;
  const float sy = ((float)py + unit24(r.y)) / (float)g.H;
  const float aspect = (float)g.W / (float)g.H;
  const float cx = (2.0f * sx - 1.0f) * sc.cam_tan_half * aspect;
  const float cy = (1.0f - 2.0f * sy) * sc.cam_tan_half;
  const f3 f = F3(sc.cam_fx, sc.cam_fy, sc.cam_fz), rr = F3(sc.cam_rx, sc.cam_ry, sc.cam_rz),
           vv = F3(sc.cam_vx, sc.cam_vy, sc.cam_vz);
  const f3 d = normalize(f + rr * cx + vv * cy);
  rays[2 * slot] = make_float4(sc.cam_px, sc.cam_py, sc.cam_pz, __uint_as_float(slot));
  rays[2 * slot + 1] = make_float4(d.x, d.y, d.z, __uint_as_float(NO_PRIM));
  beta[slot] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
  L[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  aux[2 * slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  aux[2 * slot + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

template <bool COUNT>
__global__ __launch_bounds__(TB) void k_extend(SceneView sc, const float4* __restrict__ rays,
                                               const uint32_t* __restrict__ count,
                                               float4* __restrict__ hits,
                                               uint32_t* __restrict__ spill,
                                               unsigned long long* __restrict__ stats) {
  __shared__ uint32_t stk[LDS_STACK * TB];
  const uint32_t n = *count;
  const uint32_t gtid = blockIdx.x * TB + threadIdx.x;
  Stack st{stk + threadIdx.x, spill + gtid, gridDim.x * TB, 0, 0u, false};
  WorkCount wc;
  for (uint32_t q = gtid; q < n; q += gridDim.x * TB) {
    const float4 R0 = rays[2 * q], R1 = rays[2 * q + 1];
    TraceState ts{INFINITY, NO_PRIM, 0.0f, 0.0f};
    traverse<false, COUNT>(sc, xyz(R0), xyz(R1), __float_as_uint(R1.w), NO_PRIM, NO_PRIM, st, ts,
                           wc);
    hits[q] = make_float4(ts.t, __uint_as_float(ts.prim), ts.b1, ts.b2);
  }
  if (st.spills) atomicAdd(stats + 3, (unsigned long long)st.spills);
  if (st.overflow) atomicAdd(stats + 5, 1ull);
  if (COUNT && wc.visits) atomicAdd(stats + 6, (unsigned long long)wc.visits);
  if (COUNT && wc.tests) atomicAdd(stats + 7, (unsigned long long)wc.tests);
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
__device__ __forceinline__ f3 ggx_eval(f3 f0, float alpha, f3 n, f3 wo, f3 wi, float ci,
                                       float co) {
  const f3 h = normalize(wi + wo);
  const float ch = dot(n, h);
  if (ch <= 0.0f) return F3(0.0f, 0.0f, 0.0f);
  const f3 nh = cross(n, h);
  const float a2 = alpha * alpha;
  const float den = a2 * ch * ch + dot(nh, nh);
  const float D = a2 / (3.14159265358979323846f * den * den);
  const float G = ggx_G1(a2, ci) * ggx_G1(a2, co);
  return schlick(f0, dot(wi, h)) * (D * G / (4.0f * ci * co));
}

__global__ __launch_bounds__(256) void k_shade(ChunkGeom g, SceneView sc, int b,
                                               const float4* __restrict__ rays_in,
                                               const float4* __restrict__ hits,
                                               uint32_t* __restrict__ q,
                                               float4* __restrict__ rays_out,
                                               float4* __restrict__ shadow,
                                               float4* __restrict__ beta_buf,
                                               float4* __restrict__ L_buf,
                                               float4* __restrict__ aux_buf) {
  const uint32_t n = q[Q_RAYS + b];
  uint32_t* cnt_next = q + Q_RAYS + b + 1;
  uint32_t* cnt_shadow = q + Q_SHADOW + b;
  for (uint32_t base = blockIdx.x * 256; base < n; base += gridDim.x * 256) {
    const uint32_t qi = base + threadIdx.x;
    bool cont = false, shad = false;
    uint32_t slot = 0, prim = NO_PRIM, li = 0;
    f3 x = F3(0, 0, 0), wi = F3(0, 0, 0), swi = F3(0, 0, 0), c = F3(0, 0, 0);
    float sr = 0.0f;
    if (qi < n) {
      const float4 R0 = rays_in[2 * qi], R1 = rays_in[2 * qi + 1];
      slot = __float_as_uint(R0.w);
      const f3 o = xyz(R0), d = xyz(R1);
      const float4 Hh = hits[qi];
      prim = __float_as_uint(Hh.y);
      f3 beta = xyz(beta_buf[slot]);
      f3 L = xyz(L_buf[slot]);
      if (prim == NO_PRIM) {
        L = L + mul(beta, F3(sc.env_r, sc.env_g, sc.env_b));
      } else {
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
        x = o + d * t;
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
        const DevMaterial m = sc.mats[info & PRIM_MAT_MASK];
        const int kind = (int)m.emis_kind.w;
        const f3 col = xyz(m.color_alpha);
        if (b == 0) {
          const f3 alb = kind == MRS_EMITTER ? F3(0, 0, 0) : col;
          aux_buf[2 * slot] = make_float4(alb.x, alb.y, alb.z, ns.x);
          aux_buf[2 * slot + 1] = make_float4(ns.y, ns.z, t, 0.0f);
        }
        const f3 em = xyz(m.emis_kind);
        if (front && (em.x != 0.0f || em.y != 0.0f || em.z != 0.0f) &&
            (!(info & PRIM_LISTED) || b == 0))
          L = L + mul(beta, em);
        bool alive = b != g.max_depth && kind != MRS_EMITTER && dot(ns, wo) > 0.0f;
        if (alive) {
          uint32_t P, s, pl;
          slot_pixel_sample(g, slot, P, s, pl);
          const uint4 bl = philox4x32_10(make_uint4(P, s, 1u + 2u * b, 0u), g.seed_lo, g.seed_hi);
          const uint4 bs = philox4x32_10(make_uint4(P, s, 2u + 2u * b, 0u), g.seed_lo, g.seed_hi);
          const float alpha = m.color_alpha.w;
          const float co = dot(ns, wo);
          // next-event estimation: one light chosen uniformly, area sampling
          if (sc.nlights > 0) {
            li = (uint32_t)(((uint64_t)(bl.x >> 8) * (uint64_t)sc.nlights) >> 24);
            const DevLight& lt = sc.lights[li];
            const float u1 = unit24(bl.y), u2 = unit24(bl.z);
            const f3 y = xyz(lt.corner) + xyz(lt.eu) * u1 + xyz(lt.ev) * u2;
            const f3 dv = y - x;
            const float r2 = dot(dv, dv);
            const float r = sqrtf(r2);
            const f3 w = dv * (1.0f / r);
            const float cs = dot(ns, w), cg = dot(ng, w), cl = -dot(xyz(lt.normal), w);
            if (cs > 0.0f && cg > 0.0f && cl > 0.0f) {
              const f3 f = kind == MRS_LAMBERT ? col * INV_PI : ggx_eval(col, alpha, ns, wo, w, cs, co);
              const float geo = cs * cl * ((float)sc.nlights * lt.normal.w) / r2;
              c = mul(mul(beta, f), xyz(lt.le)) * geo;
              swi = w;
              sr = r;
              shad = true;
            }
          }
          // BSDF sample
          f3 T, B;
          onb(ns, T, B);
          const float v1 = unit24(bs.x), v2 = unit24(bs.y);
          float sp, cp;
          sincospif(2.0f * v2, &sp, &cp);
          if (kind == MRS_LAMBERT) {
            const float rr = sqrtf(v1);
            wi = T * (rr * cp) + B * (rr * sp) + ns * sqrtf(1.0f - v1);
            if (dot(ng, wi) <= 0.0f) alive = false;
            beta = mul(beta, col);
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
            }
          }
          if (alive && b >= g.rr_start) {
            const float qq = fminf(0.95f, maxc(beta));
            if (!(unit24(bs.z) < qq)) alive = false;
            else beta = beta * (1.0f / qq);
          }
          beta_buf[slot] = make_float4(beta.x, beta.y, beta.z, 0.0f);
        }
        cont = alive;
      }
      L_buf[slot] = make_float4(L.x, L.y, L.z, 0.0f);
    }
    const uint32_t ri = wave_append(cont, cnt_next);
    if (cont) {
      rays_out[2 * ri] = make_float4(x.x, x.y, x.z, __uint_as_float(slot));
      rays_out[2 * ri + 1] = make_float4(wi.x, wi.y, wi.z, __uint_as_float(prim));
    }
    const uint32_t si = wave_append(shad, cnt_shadow);
    if (shad) {
      shadow[3 * si] = make_float4(x.x, x.y, x.z, __uint_as_float(slot | (li << 24)));
      shadow[3 * si + 1] = make_float4(swi.x, swi.y, swi.z, sr);
      shadow[3 * si + 2] = make_float4(c.x, c.y, c.z, __uint_as_float(prim));
    }
  }
}

template <bool COUNT>
__global__ __launch_bounds__(TB) void k_shadow(SceneView sc, const float4* __restrict__ shadow,
                                               const uint32_t* __restrict__ count,
                                               float4* __restrict__ L_buf,
                                               uint32_t* __restrict__ spill,
                                               unsigned long long* __restrict__ stats) {
  __shared__ uint32_t stk[LDS_STACK * TB];
  const uint32_t n = *count;
  const uint32_t gtid = blockIdx.x * TB + threadIdx.x;
  Stack st{stk + threadIdx.x, spill + gtid, gridDim.x * TB, 0, 0u, false};
  WorkCount wc;
  for (uint32_t q = gtid; q < n; q += gridDim.x * TB) {
    const float4 S0 = shadow[3 * q], S1 = shadow[3 * q + 1], S2 = shadow[3 * q + 2];
    const uint32_t tag = __float_as_uint(S0.w);
    const uint32_t slot = tag & 0xffffffu, li = tag >> 24;
    const DevLight& lt = sc.lights[li];
    TraceState ts{S1.w, NO_PRIM, 0.0f, 0.0f};
    const bool occ = traverse<true, COUNT>(sc, xyz(S0), xyz(S1), __float_as_uint(S2.w),
                                           (uint32_t)lt.tri0, (uint32_t)lt.tri1, st, ts, wc);
    if (!occ) {
      float4 Lv = L_buf[slot];
      Lv.x += S2.x;
      Lv.y += S2.y;
      Lv.z += S2.z;
      L_buf[slot] = Lv;
    }
  }
  if (st.spills) atomicAdd(stats + 3, (unsigned long long)st.spills);
  if (st.overflow) atomicAdd(stats + 5, 1ull);
  if (COUNT && wc.visits) atomicAdd(stats + 8, (unsigned long long)wc.visits);
  if (COUNT && wc.tests) atomicAdd(stats + 9, (unsigned long long)wc.tests);
}

template <typename T>
__global__ __launch_bounds__(256) void k_accumulate(ChunkGeom g, int32_t ns, uint32_t np,
                                                    const float4* __restrict__ L_buf,
                                                    const float4* __restrict__ aux_buf,
                                                    T* __restrict__ acc_rgb,
                                                    T* __restrict__ acc_aux,
                                                    T* __restrict__ acc_sq,
                                                    unsigned long long* __restrict__ stats) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const uint32_t pl = (uint32_t)g.p0 + i;
  T r = acc_rgb[3 * pl], gg = acc_rgb[3 * pl + 1], bb = acc_rgb[3 * pl + 2];
  T sr = acc_sq[3 * pl], sg = acc_sq[3 * pl + 1], sb = acc_sq[3 * pl + 2];
  T a[7];
  for (int c = 0; c < 7; ++c) a[c] = acc_aux[7 * pl + c];
  uint32_t bad = 0;
  for (int k = 0; k < ns; ++k) {
    const uint32_t slot = (uint32_t)k * np + i;
    float4 Lv = L_buf[slot];
    if (!(isfinite(Lv.x) && isfinite(Lv.y) && isfinite(Lv.z))) {
      Lv = make_float4(0, 0, 0, 0);
      ++bad;
    }
    r += (T)Lv.x;
    gg += (T)Lv.y;
    bb += (T)Lv.z;
    sr += (T)Lv.x * (T)Lv.x;
    sg += (T)Lv.y * (T)Lv.y;
    sb += (T)Lv.z * (T)Lv.z;
    const float4 A0 = aux_buf[2 * slot], A1 = aux_buf[2 * slot + 1];
    a[0] += (T)A0.x; a[1] += (T)A0.y; a[2] += (T)A0.z; a[3] += (T)A0.w;
    a[4] += (T)A1.x; a[5] += (T)A1.y; a[6] += (T)A1.z;
  }
  acc_rgb[3 * pl] = r; acc_rgb[3 * pl + 1] = gg; acc_rgb[3 * pl + 2] = bb;
  acc_sq[3 * pl] = sr; acc_sq[3 * pl + 1] = sg; acc_sq[3 * pl + 2] = sb;
  for (int c = 0; c < 7; ++c) acc_aux[7 * pl + c] = a[c];
  if (bad) atomicAdd(stats + 0, (unsigned long long)bad);
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(T* p, size_t n) {
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = (T)0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_resolve(uint32_t npix, int32_t spp,
                                                 const T* __restrict__ acc_rgb,
                                                 const T* __restrict__ acc_aux,
                                                 const T* __restrict__ acc_sq,
                                                 float* __restrict__ out_rgb,
                                                 float* __restrict__ out_aux,
                                                 float* __restrict__ out_sq) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npix) return;
  const T inv = (T)1 / (T)spp;
  for (int c = 0; c < 3; ++c) out_rgb[3 * i + c] = (float)(acc_rgb[3 * i + c] * inv);
  if (out_aux)
    for (int c = 0; c < 7; ++c) out_aux[7 * i + c] = (float)(acc_aux[7 * i + c] * inv);
  if (out_sq)
    for (int c = 0; c < 3; ++c) out_sq[3 * i + c] = (float)acc_sq[3 * i + c];
}

__global__ __launch_bounds__(64) void k_tally(const uint32_t* __restrict__ q, int nb,
                                              unsigned long long* __restrict__ stats,
                                              uint32_t paths) {
  if (threadIdx.x == 0) {
    unsigned long long r = 0, s = 0;
    for (int b = 0; b < nb; ++b) {
      r += q[Q_RAYS + b];
      s += q[Q_SHADOW + b];
    }
    stats[1] += r;
    stats[2] += s;
    stats[4] += paths;
  }
}

__global__ __launch_bounds__(256) void k_debug_hit(SceneView sc, int32_t n,
                                                   const float* __restrict__ o,
                                                   const float* __restrict__ d,
                                                   const int32_t* __restrict__ skip,
                                                   float* __restrict__ t_out,
                                                   int32_t* __restrict__ prim_out,
                                                   float* __restrict__ b_out,
                                                   uint32_t* __restrict__ spill) {
  __shared__ uint32_t stk[LDS_STACK * 256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  Stack st{stk + threadIdx.x, spill + i, (uint32_t)(gridDim.x * 256), 0, 0u, false};
  if (i >= n) return;
  TraceState ts{INFINITY, NO_PRIM, 0.0f, 0.0f};
  WorkCount wc;
  const uint32_t sk = skip ? (uint32_t)skip[i] : NO_PRIM;
  traverse<false, false>(sc, F3(o[3 * i], o[3 * i + 1], o[3 * i + 2]),
                         F3(d[3 * i], d[3 * i + 1], d[3 * i + 2]), sk, NO_PRIM, NO_PRIM, st, ts,
                         wc);
  t_out[i] = ts.t;
  prim_out[i] = ts.prim == NO_PRIM ? -1 : (int32_t)ts.prim;
  b_out[2 * i] = ts.b1;
  b_out[2 * i + 1] = ts.b2;
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

struct Workspace {
  size_t cap_paths = 0;
  int spill_threads = 0;
  size_t acc_pix = 0;
  float4* rays[2] = {nullptr, nullptr};
  float4* hits = nullptr;
  float4* shadow = nullptr;
  float4* beta = nullptr;
  float4* L = nullptr;
  float4* aux = nullptr;
  uint32_t* spill = nullptr;
  uint32_t* q = nullptr;
  unsigned long long* stats = nullptr;
  double* acc = nullptr;  // 13 values per pixel (rgb, aux 7, sumsq 3), FP32 or FP64
};
Workspace g_ws;
mrs_tuning g_tune = {1 << 22, 2048};
bool g_count_work = false;

template <typename T>
void hfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

mrs_status ensure_workspace(size_t paths, int threads, size_t npix) {
  if (!g_ws.q) {
    MRS_TRY_HIP(hipMalloc(&g_ws.q, sizeof(uint32_t) * Q_WORDS));
    MRS_TRY_HIP(hipMalloc(&g_ws.stats, sizeof(unsigned long long) * MRS_NUM_COUNTERS));
    MRS_TRY_HIP(hipMemset(g_ws.stats, 0, sizeof(unsigned long long) * MRS_NUM_COUNTERS));
  }
  if (paths > g_ws.cap_paths) {
    for (auto*& p : g_ws.rays) hfree(p);
    hfree(g_ws.hits);
    hfree(g_ws.shadow);
    hfree(g_ws.beta);
    hfree(g_ws.L);
    hfree(g_ws.aux);
    g_ws.cap_paths = 0;
    bool ok = hipMalloc(&g_ws.rays[0], 32 * paths) == hipSuccess &&
              hipMalloc(&g_ws.rays[1], 32 * paths) == hipSuccess &&
              hipMalloc(&g_ws.hits, 16 * paths) == hipSuccess &&
              hipMalloc(&g_ws.shadow, 48 * paths) == hipSuccess &&
              hipMalloc(&g_ws.beta, 16 * paths) == hipSuccess &&
              hipMalloc(&g_ws.L, 16 * paths) == hipSuccess &&
              hipMalloc(&g_ws.aux, 32 * paths) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      return fail(MRS_ERR_OUT_OF_MEMORY, "render: path-state allocation failed");
    }
    g_ws.cap_paths = paths;
  }
  if (threads > g_ws.spill_threads) {
    hfree(g_ws.spill);
    if (hipMalloc(&g_ws.spill, sizeof(uint32_t) * (MAX_STACK - LDS_STACK) * (size_t)threads) !=
        hipSuccess) {
      (void)hipGetLastError();
      g_ws.spill_threads = 0;
      return fail(MRS_ERR_OUT_OF_MEMORY, "render: stack spill allocation failed");
    }
    g_ws.spill_threads = threads;
  }
  if (npix > g_ws.acc_pix) {
    hfree(g_ws.acc);
    if (hipMalloc(&g_ws.acc, sizeof(double) * 13 * npix) != hipSuccess) {
      (void)hipGetLastError();
      g_ws.acc_pix = 0;
      return fail(MRS_ERR_OUT_OF_MEMORY, "render: accumulator allocation failed");
    }
    g_ws.acc_pix = npix;
  }
  return MRS_OK;
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

template <typename T>
mrs_status render_t(const mrs_scene* s, const RenderArgs& a, hipStream_t st) {
  const size_t npix = (size_t)a.ww * a.wh;
  const size_t C = (size_t)g_tune.chunk_paths;
  const int blocks = g_tune.trace_blocks;
  mrs_status rc = ensure_workspace(std::min(C, npix * (size_t)a.spp), blocks * TB, npix);
  if (rc != MRS_OK) return rc;
  T* acc_rgb = (T*)g_ws.acc;
  T* acc_aux = acc_rgb + 3 * npix;
  T* acc_sq = acc_aux + 7 * npix;
  k_zero<T><<<std::min(4096u, cdiv(13 * npix, 256)), 256, 0, st>>>(acc_rgb, 13 * npix);
  ChunkGeom g{};
  g.W = a.W;
  g.H = a.H;
  g.x0 = a.x0;
  g.y0 = a.y0;
  g.ww = a.ww;
  g.seed_lo = (uint32_t)(a.seed & 0xffffffffu);
  g.seed_hi = (uint32_t)(a.seed >> 32);
  g.max_depth = a.max_depth;
  g.rr_start = a.rr_start;
  const SceneView sc = s->view;
  // chunk plan: whole sample passes when a pass fits, else pixel ranges of one sample
  std::vector<std::pair<int, std::pair<size_t, size_t>>> plan;  // (ns, (s0 or p0, np))
  if (npix <= C) {
    const int per = (int)std::max<size_t>(1, C / npix);
    for (int s0 = 0; s0 < a.spp; s0 += per) plan.push_back({std::min(per, a.spp - s0), {(size_t)s0, npix}});
  }
  for (size_t ci = 0;; ++ci) {
    int ns;
    size_t np;
    if (npix <= C) {
      if (ci >= plan.size()) break;
      ns = plan[ci].first;
      g.s0 = (int32_t)plan[ci].second.first;
      g.p0 = 0;
      np = npix;
    } else {
      const size_t per_sample = (npix + C - 1) / C;
      const size_t sidx = ci / per_sample, part = ci % per_sample;
      if (sidx >= (size_t)a.spp) break;
      ns = 1;
      g.s0 = (int32_t)sidx;
      g.p0 = (int32_t)(part * C);
      np = std::min(C, npix - part * C);
    }
    g.np = (int32_t)np;
    const uint32_t n = (uint32_t)(np * (size_t)ns);
    const unsigned gb = std::min<unsigned>(blocks, cdiv(n, TB));
    k_reset<<<1, 256, 0, st>>>(g_ws.q, n);
    prof_begin(KID_GENERATE, st);
    k_generate<<<cdiv(n, 256), 256, 0, st>>>(g, sc, n, g_ws.rays[0], g_ws.beta, g_ws.L, g_ws.aux);
    prof_end(KID_GENERATE, st);
    for (int b = 0; b <= a.max_depth; ++b) {
      float4* rin = g_ws.rays[b & 1];
      float4* rout = g_ws.rays[(b + 1) & 1];
      prof_begin(KID_EXTEND, st);
      if (g_count_work)
        k_extend<true><<<gb, TB, 0, st>>>(sc, rin, g_ws.q + Q_RAYS + b, g_ws.hits, g_ws.spill,
                                          g_ws.stats);
      else
        k_extend<false><<<gb, TB, 0, st>>>(sc, rin, g_ws.q + Q_RAYS + b, g_ws.hits, g_ws.spill,
                                           g_ws.stats);
      prof_end(KID_EXTEND, st);
      prof_begin(KID_SHADE, st);
      k_shade<<<gb, 256, 0, st>>>(g, sc, b, rin, g_ws.hits, g_ws.q, rout, g_ws.shadow, g_ws.beta,
                                  g_ws.L, g_ws.aux);
      prof_end(KID_SHADE, st);
      if (b < a.max_depth) {
        prof_begin(KID_SHADOW, st);
        if (g_count_work)
          k_shadow<true><<<gb, TB, 0, st>>>(sc, g_ws.shadow, g_ws.q + Q_SHADOW + b, g_ws.L,
                                            g_ws.spill, g_ws.stats);
        else
          k_shadow<false><<<gb, TB, 0, st>>>(sc, g_ws.shadow, g_ws.q + Q_SHADOW + b, g_ws.L,
                                             g_ws.spill, g_ws.stats);
        prof_end(KID_SHADOW, st);
      }
    }
    prof_begin(KID_ACCUMULATE, st);
    k_accumulate<T><<<cdiv(np, 256), 256, 0, st>>>(g, ns, (uint32_t)np, g_ws.L, g_ws.aux, acc_rgb,
                                                   acc_aux, acc_sq, g_ws.stats);
    prof_end(KID_ACCUMULATE, st);
    k_tally<<<1, 64, 0, st>>>(g_ws.q, a.max_depth + 1, g_ws.stats, n);
  }
  prof_begin(KID_RESOLVE, st);
  k_resolve<T><<<cdiv(npix, 256), 256, 0, st>>>((uint32_t)npix, a.spp, acc_rgb, acc_aux, acc_sq,
                                                a.out_rgb, a.out_aux, a.out_sumsq);
  prof_end(KID_RESOLVE, st);
  MRS_TRY_HIP(hipGetLastError());
  return MRS_OK;
}

}  // namespace

mrs_status render(const mrs_scene* s, const RenderArgs& a, hipStream_t st) {
  if (a.max_depth + 2 > MAX_BOUNCE_SLOTS)
    return fail(MRS_ERR_INVALID_ARGUMENT, "render: max_depth too large");
  return a.fp64 ? render_t<double>(s, a, st) : render_t<float>(s, a, st);
}

mrs_status debug_closest_hit(const mrs_scene* s, int32_t n, const float* o, const float* d,
                             const int32_t* skip, float* t, int32_t* prim, float* b,
                             hipStream_t st) {
  if (n <= 0) return MRS_OK;
  const unsigned blocks = cdiv((size_t)n, 256);
  mrs_status rc = ensure_workspace(1, (int)(blocks * 256), 1);
  if (rc != MRS_OK) return rc;
  k_debug_hit<<<blocks, 256, 0, st>>>(s->view, n, o, d, skip, t, prim, b, g_ws.spill);
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
  if (!g_ws.stats) return MRS_OK;
  unsigned long long h[MRS_NUM_COUNTERS];
  MRS_TRY_HIP(hipMemcpyAsync(h, g_ws.stats, sizeof(h), hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < MRS_NUM_COUNTERS; ++i) out[i] = (int64_t)h[i];
  if (reset) {
    k_zero<unsigned long long><<<1, 256, 0, st>>>(g_ws.stats, MRS_NUM_COUNTERS);
    MRS_TRY_HIP(hipGetLastError());
  }
  return MRS_OK;
}

void get_tuning(mrs_tuning* t) { *t = g_tune; }

void set_count_work(bool on) { g_count_work = on; }

mrs_status set_tuning(const mrs_tuning* t) {
  if (t->chunk_paths < 256 || t->chunk_paths > (1 << 24))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: chunk_paths must be in [256, 2^24]");
  if (t->trace_blocks < 1 || t->trace_blocks > 65536)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: trace_blocks must be in [1, 65536]");
  g_tune = *t;
  return MRS_OK;
}

}  // namespace mrs
