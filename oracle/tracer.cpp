// FP64 reference path tracer -- TEST INFRASTRUCTURE ONLY.
//
// This file is the oracle that the GPU renderer is checked against.  It is
// plain, slow and written to be read next to the definitions it follows.  It
// shares no code, header or table with the GPU library; only the seeded scene
// arrays (produced by mrs_inputs) are common to both.  Only tests/, the smoke
// check and the bench's CPU-baseline leg may load it.
//
// The paper (Sec. 3.2) produces its HRLS/LRHS inputs with a Monte Carlo path
// tracer (Blender Cycles) and does not describe the tracer itself.  The
// estimator implemented here is the textbook one for the rendering equation
// (Kajiya 1986; Cook 1984 -- both cited in Sec. 1-2), with each mapping from
// uniforms to geometry taken from the published method named at its use:
//   E1  Philox4x32-10 counter-based RNG (Salmon et al., SC'11)
//   E3  pinhole camera, box pixel filter; optionally a thin lens (depth of
//       field) and a camera translated over the shutter (motion blur)
//   E4  Moller-Trumbore ray/triangle test (JGT 1997), closest hit over all
//       triangles, ties to the smaller primitive id
//   E5  shading frame, orthonormal basis of Duff et al. (JCGT 2017)
//   E7  path loop with pbrt-style depth counting
//   E8  next-event estimation on quad lights, area sampling; optionally (mis)
//       combined with BSDF sampling of the same lights by multiple importance
//       sampling with the power heuristic (Veach & Guibas, SIGGRAPH 1995)
//   E9  Lambert BRDF, cosine-weighted sampling
//   E10 GGX microfacet BRDF (Walter et al., EGSR 2007), separable Smith G,
//       Schlick Fresnel, sampling of the half vector from D(h)(n.h)
//   E11 Russian roulette
//   (offset) rays leave a vertex from a point lifted off the surface along the
//       geometric normal by an amount proportional to the point's magnitude
//       (this project's own simplified rule, inspired by the offsets of Wachter
//       & Binder, Ray Tracing Gems ch. 6, which switch to integer-ULP steps)
//   E12 per-pixel accumulation in sample order
// Arithmetic is FP64 throughout; the scene's FP32 values are promoted.
//
// Build: g++ -O2 -std=c++17 -fPIC -shared -pthread -ffp-contract=off

#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

// ----------------------------------------------------------------- vectors
struct V3 {
  double x, y, z;
};
inline V3 mk(double x, double y, double z) { return V3{x, y, z}; }
inline V3 operator+(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
inline V3 operator-(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
inline V3 operator*(V3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
inline V3 operator*(double s, V3 a) { return mk(a.x * s, a.y * s, a.z * s); }
inline V3 mul(V3 a, V3 b) { return mk(a.x * b.x, a.y * b.y, a.z * b.z); }
inline V3 neg(V3 a) { return mk(-a.x, -a.y, -a.z); }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
inline double length(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return a * (1.0 / length(a)); }
inline double maxc(V3 a) { return std::max(a.x, std::max(a.y, a.z)); }

// ----------------------------------------------------------------- E1: Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): 10 rounds of the Philox S-box on a 4x32 counter with a 2x32 key;
// the key is bumped by the Weyl constants before every round after the first.
const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {in[0], in[1], in[2], in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += PHILOX_W0;
      k[1] += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// One Philox block of four raw 32-bit words for (pixel p, sample s, block j).
// Dimension d lives in block d/4, word d%4.  Tag 0 = rendering.
struct Block {
  uint32_t w[4];
};
Block rng_block(uint64_t seed, uint32_t p, uint32_t s, uint32_t j, uint32_t tag) {
  uint32_t ctr[4] = {p, s, j, tag};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  Block b;
  philox4x32_10(ctr, key, b.w);
  return b;
}
// The 24 high bits of a word as a uniform in [0, 1 - 2^-24]; exact in FP32 and FP64.
inline double to_unit(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

// ----------------------------------------------------------------- scene
struct Material {  // 32-byte record produced by the scene generator
  int32_t kind;    // 0 Lambert, 1 GGX, 2 pure emitter
  float color[3];  // Lambert albedo or GGX F0
  float alpha;     // GGX roughness (alpha = roughness)
  float emission[3];
};
struct QuadLight {  // 56-byte record
  float corner[3], edge_u[3], edge_v[3], emission[3];
  int32_t tri[2];
};
static_assert(sizeof(Material) == 32, "material record");
static_assert(sizeof(QuadLight) == 56, "light record");

struct Tri {
  V3 v0, v1, v2;
  V3 n0, n1, n2;
  bool smooth;
  uint32_t mat;
  bool listed_light;
};
struct Light {
  V3 corner, eu, ev, le, normal;
  double area;
  int32_t tri0, tri1;
};
struct MatD {
  int kind;
  V3 color;
  double alpha;
  V3 emission;
};
struct Cam {
  V3 pos, look_at, up;
  double vfov_deg;
};

struct BvhNode {
  double lo[3], hi[3];
  int32_t left, right;  // children (internal) or -1
  int32_t first, count; // leaf primitive range in `order`
};

struct Scene {
  std::vector<Tri> tris;
  std::vector<MatD> mats;
  std::vector<Light> lights;
  V3 env;
  Cam cam;
  std::vector<BvhNode> nodes;
  std::vector<int32_t> order;
};

V3 ld3(const float* p) { return mk((double)p[0], (double)p[1], (double)p[2]); }

// ----------------------------------------------------------------- E4: intersection
// Moller & Trumbore (JGT 1997).  Edges are inclusive; det == 0 (ray parallel to
// the plane) is a miss.  Returns t or +inf.
double tri_hit(const Tri& tr, V3 o, V3 d, double* b1, double* b2) {
  const double inf = std::numeric_limits<double>::infinity();
  V3 e1 = tr.v1 - tr.v0, e2 = tr.v2 - tr.v0;
  V3 pv = cross(d, e2);
  double det = dot(e1, pv);
  if (det == 0.0 || !std::isfinite(det)) return inf;
  double inv = 1.0 / det;
  V3 tv = o - tr.v0;
  double u = dot(tv, pv) * inv;
  if (!(u >= 0.0 && u <= 1.0)) return inf;
  V3 qv = cross(tv, e1);
  double v = dot(d, qv) * inv;
  if (!(v >= 0.0 && u + v <= 1.0)) return inf;
  double t = dot(e2, qv) * inv;
  *b1 = u;
  *b2 = v;
  return t;
}

struct Hit {
  double t = std::numeric_limits<double>::infinity();
  int32_t prim = -1;
  double b1 = 0, b2 = 0;
};

// Closest hit with t > 0 over every triangle except `skip`; equal t goes to the
// smaller primitive id.  The plain definition, O(N).
Hit closest_brute(const Scene& sc, V3 o, V3 d, int32_t skip) {
  Hit h;
  for (int32_t i = 0; i < (int32_t)sc.tris.size(); ++i) {
    if (i == skip) continue;
    double b1, b2;
    double t = tri_hit(sc.tris[i], o, d, &b1, &b2);
    if (!(t > 0.0) || !std::isfinite(t)) continue;
    if (t < h.t || (t == h.t && i < h.prim)) {
      h.t = t;
      h.prim = i;
      h.b1 = b1;
      h.b2 = b2;
    }
  }
  return h;
}

// Conservative slab test: the far distance is widened by 2 ulp-scale gamma
// factors (Ize, "Robust BVH ray traversal", JCGT 2013) so that boxes are never
// culled by rounding; the exact answer then comes from the triangle tests.
bool box_hit(const BvhNode& n, V3 o, V3 inv, double tmax) {
  double t0 = 0.0, t1 = tmax;
  const double oo[3] = {o.x, o.y, o.z}, ii[3] = {inv.x, inv.y, inv.z};
  for (int a = 0; a < 3; ++a) {
    double ta = (n.lo[a] - oo[a]) * ii[a];
    double tb = (n.hi[a] - oo[a]) * ii[a];
    if (std::isnan(ta) || std::isnan(tb)) {  // 0 * inf: origin on the slab plane, parallel ray
      if (oo[a] < n.lo[a] || oo[a] > n.hi[a]) return false;
      continue;
    }
    if (ta > tb) std::swap(ta, tb);
    ta -= std::fabs(ta) * 4.0 * std::numeric_limits<double>::epsilon();
    tb += std::fabs(tb) * 4.0 * std::numeric_limits<double>::epsilon();
    t0 = std::max(t0, ta);
    t1 = std::min(t1, tb);
    if (t0 > t1) return false;
  }
  return true;
}

Hit closest_bvh(const Scene& sc, V3 o, V3 d, int32_t skip) {
  Hit h;
  if (sc.nodes.empty()) return h;
  V3 inv = mk(1.0 / d.x, 1.0 / d.y, 1.0 / d.z);
  std::vector<int32_t> stack;
  stack.push_back(0);
  while (!stack.empty()) {
    int32_t ni = stack.back();
    stack.pop_back();
    const BvhNode& n = sc.nodes[ni];
    // Ties must still be visited so the smaller primitive id can win.
    if (!box_hit(n, o, inv, h.t)) continue;
    if (n.left < 0) {
      for (int32_t k = n.first; k < n.first + n.count; ++k) {
        int32_t i = sc.order[k];
        if (i == skip) continue;
        double b1, b2;
        double t = tri_hit(sc.tris[i], o, d, &b1, &b2);
        if (!(t > 0.0) || !std::isfinite(t)) continue;
        if (t < h.t || (t == h.t && i < h.prim)) {
          h.t = t;
          h.prim = i;
          h.b1 = b1;
          h.b2 = b2;
        }
      }
    } else {
      stack.push_back(n.left);
      stack.push_back(n.right);
    }
  }
  return h;
}

// Any hit with t in (0, tmax) over all triangles except the three listed.
bool occluded(const Scene& sc, bool use_bvh, V3 o, V3 d, double tmax, int32_t s0, int32_t s1,
              int32_t s2) {
  auto test = [&](int32_t i) {
    if (i == s0 || i == s1 || i == s2) return false;
    double b1, b2;
    double t = tri_hit(sc.tris[i], o, d, &b1, &b2);
    return t > 0.0 && t < tmax;
  };
  if (!use_bvh || sc.nodes.empty()) {
    for (int32_t i = 0; i < (int32_t)sc.tris.size(); ++i)
      if (test(i)) return true;
    return false;
  }
  V3 inv = mk(1.0 / d.x, 1.0 / d.y, 1.0 / d.z);
  std::vector<int32_t> stack;
  stack.push_back(0);
  while (!stack.empty()) {
    const BvhNode& n = sc.nodes[stack.back()];
    stack.pop_back();
    if (!box_hit(n, o, inv, tmax)) continue;
    if (n.left < 0) {
      for (int32_t k = n.first; k < n.first + n.count; ++k)
        if (test(sc.order[k])) return true;
    } else {
      stack.push_back(n.left);
      stack.push_back(n.right);
    }
  }
  return false;
}

// Top-down median split over centroids, at most 4 triangles per leaf.  Only an
// accelerator for the closest-hit definition above; pinned to it by tests.
int32_t build_node(Scene& sc, std::vector<V3>& cen, int32_t first, int32_t count) {
  BvhNode n;
  for (int a = 0; a < 3; ++a) {
    n.lo[a] = std::numeric_limits<double>::infinity();
    n.hi[a] = -std::numeric_limits<double>::infinity();
  }
  for (int32_t k = first; k < first + count; ++k) {
    const Tri& t = sc.tris[sc.order[k]];
    for (V3 v : {t.v0, t.v1, t.v2}) {
      const double c[3] = {v.x, v.y, v.z};
      for (int a = 0; a < 3; ++a) {
        n.lo[a] = std::min(n.lo[a], c[a]);
        n.hi[a] = std::max(n.hi[a], c[a]);
      }
    }
  }
  n.left = n.right = -1;
  n.first = first;
  n.count = count;
  int32_t idx = (int32_t)sc.nodes.size();
  sc.nodes.push_back(n);
  if (count <= 4) return idx;
  double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
  for (int32_t k = first; k < first + count; ++k) {
    V3 c = cen[sc.order[k]];
    const double cc[3] = {c.x, c.y, c.z};
    for (int a = 0; a < 3; ++a) {
      clo[a] = std::min(clo[a], cc[a]);
      chi[a] = std::max(chi[a], cc[a]);
    }
  }
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  int32_t mid = first + count / 2;
  auto key = [&](int32_t i) {
    V3 c = cen[i];
    return axis == 0 ? c.x : (axis == 1 ? c.y : c.z);
  };
  std::nth_element(sc.order.begin() + first, sc.order.begin() + mid,
                   sc.order.begin() + first + count, [&](int32_t a, int32_t b) {
                     double ka = key(a), kb = key(b);
                     return ka < kb || (ka == kb && a < b);
                   });
  int32_t l = build_node(sc, cen, first, mid - first);
  int32_t r = build_node(sc, cen, mid, first + count - mid);
  sc.nodes[idx].left = l;
  sc.nodes[idx].right = r;
  return idx;
}

// ----------------------------------------------------------------- E5: shading frame
// Orthonormal basis around unit n (Duff et al., "Building an orthonormal basis,
// revisited", JCGT 2017), with sign(0) = +1.
void onb(V3 n, V3* T, V3* B) {
  double s = n.z >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (s + n.z);
  double b = n.x * n.y * a;
  *T = mk(1.0 + s * n.x * n.x * a, s * b, -s * n.x);
  *B = mk(b, s + n.y * n.y * a, -n.y);
}
inline V3 to_world(V3 l, V3 T, V3 B, V3 n) { return T * l.x + B * l.y + n * l.z; }

// ----------------------------------------------------------------- E9: Lambert
// Cosine-weighted hemisphere sampling via the concentric-free polar map:
// r = sqrt(u1), phi = 2 pi u2, z = sqrt(1 - u1).  pdf = cos/pi, so the
// estimator weight f cos / pdf is exactly the albedo.
V3 sample_cosine(double u1, double u2) {
  double r = std::sqrt(u1), phi = 2.0 * M_PI * u2;
  return mk(r * std::cos(phi), r * std::sin(phi), std::sqrt(1.0 - u1));
}

// ----------------------------------------------------------------- E10: GGX
// Walter, Marschner, Li, Torrance, "Microfacet models for refraction through
// rough surfaces" (EGSR 2007): GGX distribution D, separable Smith shadowing
// G = G1(wi) G1(wo), Schlick's Fresnel with F0 colour; half vector sampled
// with density D(h)(n.h).
double ggx_D(double alpha, double cos_h) {
  if (cos_h <= 0.0) return 0.0;
  double a2 = alpha * alpha;
  double den = cos_h * cos_h * (a2 - 1.0) + 1.0;
  return a2 / (M_PI * den * den);
}
double ggx_G1(double alpha, double cos_v) {
  if (cos_v <= 0.0) return 0.0;
  double a2 = alpha * alpha;
  return 2.0 * cos_v / (cos_v + std::sqrt(a2 + (1.0 - a2) * cos_v * cos_v));
}
V3 schlick(V3 f0, double c) {
  double m = 1.0 - c;
  double m5 = m * m * m * m * m;
  return mk(f0.x + (1.0 - f0.x) * m5, f0.y + (1.0 - f0.y) * m5, f0.z + (1.0 - f0.z) * m5);
}
// Half vector in the local frame (z = normal).
V3 sample_ggx_h(double alpha, double u1, double u2) {
  double a2 = alpha * alpha;
  double cos2 = (1.0 - u1) / (1.0 + (a2 - 1.0) * u1);
  double cost = std::sqrt(cos2), sint = std::sqrt(std::max(0.0, 1.0 - cos2));
  double phi = 2.0 * M_PI * u2;
  return mk(sint * std::cos(phi), sint * std::sin(phi), cost);
}
// Density (solid angle) of the reflected direction wi when the half vector is
// sampled with density D(h)(n.h): D(h)(n.h) / (4 wo.h).
double ggx_pdf(double alpha, V3 n, V3 wo, V3 wi) {
  V3 h = normalize(wi + wo);
  double ch = dot(n, h), oh = dot(wo, h);
  if (ch <= 0.0 || oh <= 0.0) return 0.0;
  return ggx_D(alpha, ch) * ch / (4.0 * oh);
}
// f(wo, wi) for the GGX lobe; n is the shading normal.
V3 ggx_eval(const MatD& m, V3 n, V3 wo, V3 wi) {
  double cos_i = dot(n, wi), cos_o = dot(n, wo);
  if (cos_i <= 0.0 || cos_o <= 0.0) return mk(0, 0, 0);
  V3 h = normalize(wi + wo);
  double D = ggx_D(m.alpha, dot(n, h));
  double G = ggx_G1(m.alpha, cos_i) * ggx_G1(m.alpha, cos_o);
  V3 F = schlick(m.color, dot(wi, h));
  return F * (D * G / (4.0 * cos_i * cos_o));
}

// ----------------------------------------------------------------- E3: camera
// Pinhole camera; (sx, sy) in [0,1)^2 across the image, row 0 at the top.
void camera_ray(const Cam& c, int W, int H, double x, double y, V3* o, V3* d) {
  V3 f = normalize(c.look_at - c.pos);
  V3 r = normalize(cross(f, c.up));
  V3 v = cross(r, f);
  double th = std::tan(0.5 * c.vfov_deg * M_PI / 180.0);
  double aspect = (double)W / (double)H;
  double sx = x / W, sy = y / H;
  *o = c.pos;
  *d = normalize(f + r * ((2.0 * sx - 1.0) * th * aspect) + v * ((1.0 - 2.0 * sy) * th));
}

// Camera effects of one render: a thin lens of radius lens_r focused on the
// plane at distance focus along the view axis (the pinhole ray through the
// pixel point meets that plane at F; the ray leaves from a point of the lens
// disk towards F), and a camera translated by motion * tau, tau in [0, 1) the
// shutter time of the sample.  Zero radius and zero motion give the pinhole.
struct CamFx {
  double lens_r, focus;
  V3 motion;
};

void camera_ray_fx(const Cam& c, const CamFx& fx, int W, int H, double x, double y, double ul0,
                   double ul1, double tau, V3* o, V3* d) {
  camera_ray(c, W, H, x, y, o, d);
  *o = *o + fx.motion * tau;
  if (fx.lens_r > 0.0) {
    V3 f = normalize(c.look_at - c.pos);
    V3 r = normalize(cross(f, c.up));
    V3 v = cross(r, f);
    V3 F = *o + *d * (fx.focus / dot(*d, f));
    double rho = fx.lens_r * std::sqrt(ul0), phi = 2.0 * M_PI * ul1;
    V3 lens = *o + r * (rho * std::cos(phi)) + v * (rho * std::sin(phi));
    *o = lens;
    *d = normalize(F - lens);
  }
}

// ----------------------------------------------------------------- E7: one path
struct PathOut {
  V3 L;
  double aux[7];
  int64_t segments;
  // Render layers (Sec. 3.1, Eqs. 1-2, without subsurface and transmission):
  // the radiance emitted towards the camera at the first vertex (emission or
  // environment) and the lobe of that vertex (0 none, 1 Lambert = diffuse,
  // 2 GGX = glossy), which owns the rest of the path's radiance.
  V3 le0;
  int lobe;
};

// Power-heuristic weight (exponent 2) of a strategy with density a against one
// with density b.
double power_weight(double a, double b) { return a * a / (a * a + b * b); }

// Density (solid angle, from the NEE strategy) of reaching light `lt` along a
// direction that meets it at distance t with cosine cl at the light.
double light_pdf(const Scene& sc, const Light& lt, double t, double cl) {
  return t * t / ((double)sc.lights.size() * lt.area * cl);
}

PathOut trace_path(const Scene& sc, bool use_bvh, int W, int H, int px, int py, int s,
                   int max_depth, int rr_start, uint64_t seed, bool mis, const CamFx& fx) {
  PathOut out;
  out.L = mk(0, 0, 0);
  for (int i = 0; i < 7; ++i) out.aux[i] = 0.0;
  out.segments = 0;
  out.le0 = mk(0, 0, 0);
  out.lobe = 0;
  const uint32_t p = (uint32_t)(py * W + px);
  // d0, d1: pixel jitter (box filter); d2, d3: lens sample; the shutter time
  // is word 0 of the block with counter (p, s, 0, 4) (drawn only for a moving
  // camera).
  Block b0 = rng_block(seed, p, (uint32_t)s, 0, 0);
  const bool moving = fx.motion.x != 0.0 || fx.motion.y != 0.0 || fx.motion.z != 0.0;
  const double tau = moving ? to_unit(rng_block(seed, p, (uint32_t)s, 0, 4).w[0]) : 0.0;
  V3 o, d;
  camera_ray_fx(sc.cam, fx, W, H, px + to_unit(b0.w[0]), py + to_unit(b0.w[1]), to_unit(b0.w[2]),
                to_unit(b0.w[3]), tau, &o, &d);
  V3 beta = mk(1, 1, 1), L = mk(0, 0, 0);
  double bsdf_pdf = 0.0;  // density of the BSDF sample that led to this vertex (mis)
  int32_t skip = -1;
  const int nL = (int)sc.lights.size();
  for (int b = 0;; ++b) {
    Hit h = use_bvh ? closest_bvh(sc, o, d, skip) : closest_brute(sc, o, d, skip);
    out.segments++;
    if (h.prim < 0) {  // miss: constant environment
      L = L + mul(beta, sc.env);
      if (b == 0) out.le0 = L;
      break;
    }
    const Tri& tr = sc.tris[h.prim];
    const MatD& m = sc.mats[tr.mat];
    V3 x = o + d * h.t;
    V3 wo = neg(d);
    V3 ng = normalize(cross(tr.v1 - tr.v0, tr.v2 - tr.v0));
    V3 ns = ng;
    if (tr.smooth)
      ns = normalize(tr.n0 * (1.0 - h.b1 - h.b2) + tr.n1 * h.b1 + tr.n2 * h.b2);
    bool front = dot(ng, wo) > 0.0;
    if (!front) {  // two-sided BSDF: shade on the side the ray arrives from
      ng = neg(ng);
      ns = neg(ns);
    }
    // Origin of the rays leaving this vertex: the hit point lifted along the
    // geometric normal on the arrival side by 2^-16 * max(1, |x|_inf).  This is
    // the project's own reading (the paper's renderer is not described): a
    // single offset proportional to the point's magnitude, simpler than the
    // offsets of Wachter & Binder (Ray Tracing Gems, ch. 6), which move the
    // point by integer ULPs away from the origin.  Every ray that leaves (NEE
    // and BSDF) has n_g . wi > 0, so it starts on the correct side.
    const double lift = std::ldexp(std::max(1.0, std::max(std::fabs(x.x), std::max(std::fabs(x.y),
                                                                       std::fabs(x.z)))), -16);
    const V3 xo = x + ng * lift;
    if (b == 0) {  // E6: first-hit feature buffers
      V3 alb = m.kind == 2 ? mk(0, 0, 0) : m.color;
      out.aux[0] = alb.x;
      out.aux[1] = alb.y;
      out.aux[2] = alb.z;
      out.aux[3] = ns.x;
      out.aux[4] = ns.y;
      out.aux[5] = ns.z;
      out.aux[6] = h.t;
    }
    // Emission from front faces.  Listed quad lights count only when seen
    // directly (b = 0): afterwards next-event estimation accounts for them --
    // or, with mis, BSDF sampling shares them with next-event estimation,
    // weighted by the power heuristic against the light-sampling density.
    if (front && (m.emission.x != 0.0 || m.emission.y != 0.0 || m.emission.z != 0.0)) {
      if (!tr.listed_light || b == 0) {
        L = L + mul(beta, m.emission);
      } else if (mis) {
        const Light* lt = nullptr;
        for (const Light& l : sc.lights)
          if (l.tri0 == h.prim || l.tri1 == h.prim) {
            lt = &l;
            break;
          }
        const double cl = dot(lt->normal, wo);
        if (cl > 0.0) {
          const double w = power_weight(bsdf_pdf, light_pdf(sc, *lt, h.t, cl));
          L = L + mul(beta, m.emission) * w;
        }
      }
    }
    if (b == 0) {
      out.le0 = L;
      out.lobe = m.kind == 0 ? 1 : (m.kind == 1 ? 2 : 0);
    }
    if (b == max_depth || m.kind == 2) break;
    if (dot(ns, wo) <= 0.0) break;  // shading normal faces away from the viewer
    const int base_block = 1 + 2 * b;  // dims 4+8b .. 4+8b+7
    Block bl = rng_block(seed, p, (uint32_t)s, (uint32_t)base_block, 0);
    Block bs = rng_block(seed, p, (uint32_t)s, (uint32_t)base_block + 1, 0);
    // ---- E8: next-event estimation, one uniformly chosen quad light
    if (nL > 0) {
      // floor(u * nL) taken on the 24-bit integer behind u: exact.
      int li = (int)(((uint64_t)(bl.w[0] >> 8) * (uint64_t)nL) >> 24);
      const Light& lt = sc.lights[li];
      double u1 = to_unit(bl.w[1]), u2 = to_unit(bl.w[2]);
      V3 y = lt.corner + lt.eu * u1 + lt.ev * u2;
      V3 dv = y - xo;
      double r2 = dot(dv, dv);
      double r = std::sqrt(r2);
      V3 wi = dv * (1.0 / r);
      double cs = dot(ns, wi), cg = dot(ng, wi), cl = -dot(lt.normal, wi);
      if (cs > 0.0 && cg > 0.0 && cl > 0.0) {
        if (!occluded(sc, use_bvh, xo, wi, r, h.prim, lt.tri0, lt.tri1)) {
          V3 f = m.kind == 0 ? m.color * (1.0 / M_PI) : ggx_eval(m, ns, wo, wi);
          double pdfA = 1.0 / ((double)nL * lt.area);
          V3 c = mul(mul(beta, f), lt.le) * (cs * cl / (r2 * pdfA));
          if (mis) {
            const double pb = m.kind == 0 ? cs / M_PI : ggx_pdf(m.alpha, ns, wo, wi);
            c = c * power_weight(light_pdf(sc, lt, r, cl), pb);
          }
          L = L + c;
        }
        out.segments++;
      }
    }
    // ---- BSDF sampling
    V3 T, B;
    onb(ns, &T, &B);
    double v1 = to_unit(bs.w[0]), v2 = to_unit(bs.w[1]);
    V3 wi;
    if (m.kind == 0) {
      wi = to_world(sample_cosine(v1, v2), T, B, ns);
      if (dot(ng, wi) <= 0.0) break;
      beta = mul(beta, m.color);
      bsdf_pdf = dot(ns, wi) / M_PI;
    } else {
      V3 hh = to_world(sample_ggx_h(m.alpha, v1, v2), T, B, ns);
      double oh = dot(wo, hh);
      wi = hh * (2.0 * oh) - wo;
      double ci = dot(ns, wi);
      if (ci <= 0.0 || dot(ng, wi) <= 0.0) break;
      double co = dot(ns, wo), ch = dot(ns, hh);
      double G = ggx_G1(m.alpha, ci) * ggx_G1(m.alpha, co);
      V3 F = schlick(m.color, oh);
      beta = mul(beta, F * (G * oh / (co * ch)));
      bsdf_pdf = ggx_D(m.alpha, ch) * ch / (4.0 * oh);
    }
    // ---- E11: Russian roulette from vertex rr_start on
    if (b >= rr_start) {
      double q = std::min(0.95, maxc(beta));
      if (!(to_unit(bs.w[2]) < q)) break;
      beta = beta * (1.0 / q);
    }
    o = xo;
    d = wi;
    skip = h.prim;
  }
  out.L = L;
  return out;
}

Scene* make_scene(int32_t ntris, const float* verts, const float* normals, const uint32_t* tmat,
                  const uint32_t* tflags, int32_t nmat, const void* mats, int32_t nlights,
                  const void* lights, const float* env, const float* cam) {
  Scene* sc = new Scene();
  const Material* M = (const Material*)mats;
  for (int i = 0; i < nmat; ++i) {
    MatD m;
    m.kind = M[i].kind;
    m.color = ld3(M[i].color);
    m.alpha = M[i].alpha;
    m.emission = ld3(M[i].emission);
    sc->mats.push_back(m);
  }
  sc->tris.resize(ntris);
  for (int i = 0; i < ntris; ++i) {
    Tri& t = sc->tris[i];
    t.v0 = ld3(verts + 9 * i);
    t.v1 = ld3(verts + 9 * i + 3);
    t.v2 = ld3(verts + 9 * i + 6);
    t.smooth = normals && (tflags[i] & 1u);
    if (t.smooth) {
      t.n0 = ld3(normals + 9 * i);
      t.n1 = ld3(normals + 9 * i + 3);
      t.n2 = ld3(normals + 9 * i + 6);
    }
    t.mat = tmat[i];
    t.listed_light = false;
  }
  const QuadLight* Q = (const QuadLight*)lights;
  for (int i = 0; i < nlights; ++i) {
    Light l;
    l.corner = ld3(Q[i].corner);
    l.eu = ld3(Q[i].edge_u);
    l.ev = ld3(Q[i].edge_v);
    l.le = ld3(Q[i].emission);
    V3 c = cross(l.eu, l.ev);
    l.area = length(c);
    l.normal = c * (1.0 / l.area);
    l.tri0 = Q[i].tri[0];
    l.tri1 = Q[i].tri[1];
    if (l.tri0 >= 0 && l.tri0 < ntris) sc->tris[l.tri0].listed_light = true;
    if (l.tri1 >= 0 && l.tri1 < ntris) sc->tris[l.tri1].listed_light = true;
    sc->lights.push_back(l);
  }
  sc->env = ld3(env);
  sc->cam.pos = ld3(cam);
  sc->cam.look_at = ld3(cam + 3);
  sc->cam.up = ld3(cam + 6);
  sc->cam.vfov_deg = cam[9];
  if (ntris > 0) {
    std::vector<V3> cen(ntris);
    for (int i = 0; i < ntris; ++i)
      cen[i] = (sc->tris[i].v0 + sc->tris[i].v1 + sc->tris[i].v2) * (1.0 / 3.0);
    sc->order.resize(ntris);
    for (int i = 0; i < ntris; ++i) sc->order[i] = i;
    build_node(*sc, cen, 0, ntris);
  }
  return sc;
}

}  // namespace

extern "C" {

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

void* orc_scene_create(int32_t ntris, const float* verts, const float* normals,
                       const uint32_t* tmat, const uint32_t* tflags, int32_t nmat,
                       const void* mats, int32_t nlights, const void* lights, const float* env,
                       const float* cam) {
  return make_scene(ntris, verts, normals, tmat, tflags, nmat, mats, nlights, lights, env, cam);
}

void orc_scene_destroy(void* s) { delete (Scene*)s; }

int32_t orc_bvh_nodes(void* s) { return (int32_t)((Scene*)s)->nodes.size(); }

// Closest hit for n rays (origins/directions as FP64 xyz triples).
void orc_closest_hit(void* s, int32_t use_bvh, int32_t n, const double* o, const double* d,
                     const int32_t* skip, double* t_out, int32_t* prim_out, double* b_out) {
  const Scene& sc = *(const Scene*)s;
  for (int i = 0; i < n; ++i) {
    V3 oo = mk(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
    V3 dd = mk(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
    int32_t sk = skip ? skip[i] : -1;
    Hit h = use_bvh ? closest_bvh(sc, oo, dd, sk) : closest_brute(sc, oo, dd, sk);
    t_out[i] = h.t;
    prim_out[i] = h.prim;
    b_out[2 * i] = h.b1;
    b_out[2 * i + 1] = h.b2;
  }
}

void orc_camera_ray(void* s, int32_t W, int32_t H, double x, double y, double* o, double* d) {
  V3 oo, dd;
  camera_ray(((Scene*)s)->cam, W, H, x, y, &oo, &dd);
  o[0] = oo.x; o[1] = oo.y; o[2] = oo.z;
  d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
}

// camfx: lens radius, focus distance, motion xyz (NULL: pinhole, no motion).
static CamFx make_fx(const double* camfx) {
  CamFx fx;
  fx.lens_r = camfx ? camfx[0] : 0.0;
  fx.focus = camfx ? camfx[1] : 0.0;
  fx.motion = camfx ? mk(camfx[2], camfx[3], camfx[4]) : mk(0, 0, 0);
  return fx;
}

void orc_camera_ray_fx(void* s, int32_t W, int32_t H, double x, double y, double ul0, double ul1,
                       double tau, const double* camfx, double* o, double* d) {
  V3 oo, dd;
  camera_ray_fx(((Scene*)s)->cam, make_fx(camfx), W, H, x, y, ul0, ul1, tau, &oo, &dd);
  o[0] = oo.x; o[1] = oo.y; o[2] = oo.z;
  d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
}

void orc_onb(const double* n, double* T, double* B) {
  V3 t, b;
  onb(mk(n[0], n[1], n[2]), &t, &b);
  T[0] = t.x; T[1] = t.y; T[2] = t.z;
  B[0] = b.x; B[1] = b.y; B[2] = b.z;
}

void orc_sample_cosine(double u1, double u2, double* out) {
  V3 v = sample_cosine(u1, u2);
  out[0] = v.x; out[1] = v.y; out[2] = v.z;
}

double orc_ggx_D(double alpha, double cos_h) { return ggx_D(alpha, cos_h); }
double orc_ggx_G1(double alpha, double cos_v) { return ggx_G1(alpha, cos_v); }

void orc_sample_ggx_h(double alpha, double u1, double u2, double* out) {
  V3 v = sample_ggx_h(alpha, u1, u2);
  out[0] = v.x; out[1] = v.y; out[2] = v.z;
}

void orc_ggx_eval(double alpha, const double* f0, const double* n, const double* wo,
                  const double* wi, double* out) {
  MatD m;
  m.kind = 1;
  m.alpha = alpha;
  m.color = mk(f0[0], f0[1], f0[2]);
  m.emission = mk(0, 0, 0);
  V3 f = ggx_eval(m, mk(n[0], n[1], n[2]), mk(wo[0], wo[1], wo[2]), mk(wi[0], wi[1], wi[2]));
  out[0] = f.x; out[1] = f.y; out[2] = f.z;
}

// Render: for each requested pixel (all W*H when pixels == NULL), the mean over
// spp samples of the path radiance (E12: summed in sample order) and of the
// first-hit features.  out_sumsq (optional) receives sum_s L^2 per channel.
// mis = 1 combines next-event estimation and BSDF sampling of the quad lights;
// camfx (or NULL) = lens radius, focus distance, camera motion xyz.
// counters[0] = non-finite samples replaced by 0, counters[1] = rays traced.
// out_layers (optional, 9 per pixel): the means of the emission seen at the
// first vertex, and of the rest of the radiance of the samples whose first
// vertex is Lambert (diffuse) and GGX (glossy); the three add up to rgb.
int32_t orc_render(void* s, int32_t W, int32_t H, int32_t spp, int32_t max_depth,
                   int32_t rr_start, uint64_t seed, int32_t npix, const int32_t* pixels,
                   double* out_rgb, double* out_aux, double* out_sumsq, int32_t nthreads,
                   int32_t use_bvh, int32_t mis, const double* camfx, int64_t* counters,
                   double* out_layers) {
  const Scene& sc = *(const Scene*)s;
  if (W <= 0 || H <= 0 || spp <= 0 || max_depth < 0 || (mis != 0 && mis != 1)) return 1;
  const CamFx fx = make_fx(camfx);
  if (fx.lens_r < 0.0 || (fx.lens_r > 0.0 && !(fx.focus > 0.0))) return 1;
  int64_t n = pixels ? npix : (int64_t)W * H;
  std::atomic<int64_t> next(0), nonfinite(0), segs(0);
  auto work = [&]() {
    for (;;) {
      int64_t k0 = next.fetch_add(64);
      if (k0 >= n) break;
      int64_t k1 = std::min(n, k0 + 64);
      for (int64_t k = k0; k < k1; ++k) {
        int64_t pix = pixels ? pixels[k] : k;
        int px = (int)(pix % W), py = (int)(pix / W);
        double sum[3] = {0, 0, 0}, sq[3] = {0, 0, 0}, aux[7] = {0, 0, 0, 0, 0, 0, 0};
        double lay[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        int64_t lseg = 0;
        for (int si = 0; si < spp; ++si) {
          PathOut po = trace_path(sc, use_bvh != 0, W, H, px, py, si, max_depth, rr_start, seed,
                                  mis != 0, fx);
          lseg += po.segments;
          double l[3] = {po.L.x, po.L.y, po.L.z};
          double e[3] = {po.le0.x, po.le0.y, po.le0.z};
          if (!(std::isfinite(l[0]) && std::isfinite(l[1]) && std::isfinite(l[2]))) {
            l[0] = l[1] = l[2] = 0.0;
            e[0] = e[1] = e[2] = 0.0;
            nonfinite++;
          }
          // layers: emission at the first vertex; the rest to its lobe
          for (int c = 0; c < 3; ++c) {
            lay[c] += e[c];
            if (po.lobe > 0) lay[3 * po.lobe + c] += l[c] - e[c];
          }
          for (int c = 0; c < 3; ++c) {
            sum[c] += l[c];
            sq[c] += l[c] * l[c];
          }
          for (int c = 0; c < 7; ++c) aux[c] += po.aux[c];
        }
        segs += lseg;
        for (int c = 0; c < 3; ++c) out_rgb[3 * k + c] = sum[c] / spp;
        if (out_sumsq)
          for (int c = 0; c < 3; ++c) out_sumsq[3 * k + c] = sq[c];
        if (out_aux)
          for (int c = 0; c < 7; ++c) out_aux[7 * k + c] = aux[c] / spp;
        if (out_layers)
          for (int c = 0; c < 9; ++c) out_layers[9 * k + c] = lay[c] / spp;
      }
    }
  };
  int nt = std::max(1, (int)nthreads);
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (counters) {
    counters[0] = nonfinite.load();
    counters[1] = segs.load();
  }
  return 0;
}

}  // extern "C"
