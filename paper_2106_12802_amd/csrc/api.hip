// Host side of the C ABI: validation, scene upload, stream and error state.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mrs_internal.hpp"

namespace mrs {

namespace {
thread_local std::string t_error;
thread_local hipStream_t t_stream = nullptr;
}  // namespace

const std::string& t_error_ref() { return t_error; }
void set_stream(hipStream_t s) { t_stream = s; }

void set_error(const std::string& msg) { t_error = msg; }

mrs_status fail(mrs_status st, const std::string& msg) {
  t_error = msg;
  return st;
}

mrs_status check_hip(hipError_t e, const char* what) {
  t_error = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
  return e == hipErrorOutOfMemory ? MRS_ERR_OUT_OF_MEMORY : MRS_ERR_DEVICE;
}

hipStream_t current_stream() { return t_stream; }

}  // namespace mrs

using namespace mrs;

namespace {

struct D3 {
  double x, y, z;
};
D3 d3(const float* p) { return {p[0], p[1], p[2]}; }
D3 sub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
D3 crs(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double len(D3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }
D3 nrm(D3 a) {
  double l = len(a);
  return {a.x / l, a.y / l, a.z / l};
}
float bits_to_float(uint32_t u) {
  float f;
  std::memcpy(&f, &u, sizeof f);
  return f;
}
bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

template <typename T>
mrs_status upload(T** dst, const void* src, size_t bytes) {
  if (bytes == 0) {
    *dst = nullptr;
    return MRS_OK;
  }
  if (hipMalloc((void**)dst, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_scene_create: device allocation failed");
  }
  MRS_TRY_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return MRS_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_scene(mrs_scene* s) {
  dfree(s->d_tri_src);
  dfree(s->d_prim_ng);
  dfree(s->d_prim_n);
  dfree(s->d_leaf_tri);
  dfree(s->d_nodes);
  dfree(s->d_nodes4);
  dfree(s->d_nodes4q);
  dfree(s->d_morton);
  dfree(s->d_leaf_prim);
  dfree(s->d_mats);
  dfree(s->d_lights);
}

mrs_status scene_create_impl(const mrs_scene_desc* d, mrs_scene* s) {
  const int n = d->num_tris;
  std::vector<float4> tri(3 * (size_t)n), ng(n), pn;
  const bool has_n = d->normals != nullptr;
  if (has_n) pn.resize(3 * (size_t)n);
  std::vector<uint8_t> listed(n, 0);
  for (int i = 0; i < d->num_lights; ++i) {
    listed[d->lights[i].tri[0]] = 1;
    listed[d->lights[i].tri[1]] = 1;
  }
  for (int i = 0; i < n; ++i) {
    const float* v = d->vertices + 9 * (size_t)i;
    for (int k = 0; k < 3; ++k) tri[3 * i + k] = make_float4(v[3 * k], v[3 * k + 1], v[3 * k + 2], 0.f);
    D3 g = nrm(crs(sub(d3(v + 3), d3(v)), sub(d3(v + 6), d3(v))));
    const uint32_t flags = d->tri_flags ? d->tri_flags[i] : 0u;
    const bool smooth = has_n && (flags & MRS_TRI_SMOOTH);
    uint32_t info = d->tri_material[i] | (smooth ? PRIM_SMOOTH : 0u) | (listed[i] ? PRIM_LISTED : 0u);
    ng[i] = make_float4((float)g.x, (float)g.y, (float)g.z, bits_to_float(info));
    if (has_n) {
      const float* nn = d->normals + 9 * (size_t)i;
      for (int k = 0; k < 3; ++k)
        pn[3 * i + k] = make_float4(nn[3 * k], nn[3 * k + 1], nn[3 * k + 2], 0.f);
    }
  }
  std::vector<DevMaterial> mats(d->num_materials);
  for (int i = 0; i < d->num_materials; ++i) {
    const mrs_material& m = d->materials[i];
    mats[i].color_alpha = make_float4(m.color[0], m.color[1], m.color[2], m.alpha);
    mats[i].emis_kind = make_float4(m.emission[0], m.emission[1], m.emission[2], (float)m.kind);
  }
  std::vector<DevLight> lights(d->num_lights);
  for (int i = 0; i < d->num_lights; ++i) {
    const mrs_quad_light& l = d->lights[i];
    D3 c = crs(d3(l.edge_u), d3(l.edge_v));
    double area = len(c);
    D3 nn = nrm(c);
    DevLight& o = lights[i];
    o.corner = make_float4(l.corner[0], l.corner[1], l.corner[2], 0.f);
    o.eu = make_float4(l.edge_u[0], l.edge_u[1], l.edge_u[2], 0.f);
    o.ev = make_float4(l.edge_v[0], l.edge_v[1], l.edge_v[2], 0.f);
    o.le = make_float4(l.emission[0], l.emission[1], l.emission[2], 0.f);
    o.normal = make_float4((float)nn.x, (float)nn.y, (float)nn.z, (float)area);
    o.tri0 = l.tri[0];
    o.tri1 = l.tri[1];
    o.pad0 = o.pad1 = 0;
  }
  mrs_status rc;
  if ((rc = upload(&s->d_tri_src, tri.data(), sizeof(float4) * tri.size())) != MRS_OK) return rc;
  if ((rc = upload(&s->d_prim_ng, ng.data(), sizeof(float4) * ng.size())) != MRS_OK) return rc;
  if (has_n && (rc = upload(&s->d_prim_n, pn.data(), sizeof(float4) * pn.size())) != MRS_OK)
    return rc;
  if ((rc = upload(&s->d_mats, mats.data(), sizeof(DevMaterial) * mats.size())) != MRS_OK) return rc;
  if ((rc = upload(&s->d_lights, lights.data(), sizeof(DevLight) * lights.size())) != MRS_OK)
    return rc;
  if (n > 0) {
    bool ok = hipMalloc(&s->d_leaf_tri, sizeof(float4) * 3 * (size_t)n) == hipSuccess &&
              hipMalloc(&s->d_morton, sizeof(uint32_t) * n) == hipSuccess &&
              hipMalloc(&s->d_leaf_prim, sizeof(uint32_t) * n) == hipSuccess &&
              (n < 2 || hipMalloc(&s->d_nodes, sizeof(float4) * 4 * (size_t)(n - 1)) == hipSuccess);
    if (!ok) {
      (void)hipGetLastError();
      return fail(MRS_ERR_OUT_OF_MEMORY, "mrs_scene_create: BVH allocation failed");
    }
  }
  s->ntris = n;
  s->nmats = d->num_materials;
  s->nlights = d->num_lights;
  // camera basis in FP64, rounded once
  const mrs_camera& cam = d->camera;
  D3 f = nrm(sub(d3(cam.look_at), d3(cam.pos)));
  D3 r = nrm(crs(f, d3(cam.up)));
  D3 v = crs(r, f);
  SceneView& sv = s->view;
  sv.ntris = n;
  sv.nlights = d->num_lights;
  sv.nodes = nullptr;  // BVH4, set by mrs_build_bvh
  sv.nodes_q = nullptr;
  sv.nnodes = 0;
  sv.leaf_tri = s->d_leaf_tri;
  sv.prim_ng = s->d_prim_ng;
  sv.prim_n = s->d_prim_n;
  sv.mats = s->d_mats;
  sv.lights = s->d_lights;
  sv.env_r = d->env[0];
  sv.env_g = d->env[1];
  sv.env_b = d->env[2];
  sv.cam_px = cam.pos[0];
  sv.cam_py = cam.pos[1];
  sv.cam_pz = cam.pos[2];
  sv.cam_fx = (float)f.x; sv.cam_fy = (float)f.y; sv.cam_fz = (float)f.z;
  sv.cam_rx = (float)r.x; sv.cam_ry = (float)r.y; sv.cam_rz = (float)r.z;
  sv.cam_vx = (float)v.x; sv.cam_vy = (float)v.y; sv.cam_vz = (float)v.z;
  sv.cam_tan_half = (float)std::tan(0.5 * (double)cam.vfov_deg * M_PI / 180.0);
  return MRS_OK;
}

}  // namespace

extern "C" {

const char* mrs_last_error(void) { return mrs::t_error_ref().c_str(); }

mrs_status mrs_set_stream(void* hip_stream) {
  mrs::set_stream((hipStream_t)hip_stream);
  return MRS_OK;
}

mrs_status mrs_sync(void) {
  hipError_t e = hipStreamSynchronize(current_stream());
  if (e != hipSuccess) return check_hip(e, "mrs_sync");
  return MRS_OK;
}

mrs_status mrs_scene_create(const mrs_scene_desc* d, mrs_scene** out) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: out is NULL");
  *out = nullptr;
  if (!d) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: desc is NULL");
  const int n = d->num_tris;
  if (n < 0 || n > MAX_TRIS)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: num_tris must be in [0, 2^24 - 2]");
  if (n > 0 && (!d->vertices || !d->tri_material))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: vertices/tri_material NULL");
  if (d->num_materials < 0 || (d->num_materials > 0 && !d->materials) ||
      d->num_materials > (1 << 24))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: bad materials");
  if (d->num_lights < 0 || d->num_lights > MAX_LIGHTS || (d->num_lights > 0 && !d->lights))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: num_lights must be in [0, 255]");
  for (int i = 0; i < d->num_materials; ++i) {
    const mrs_material& m = d->materials[i];
    if (m.kind < 0 || m.kind > 2 || !finite3(m.color) || !finite3(m.emission) ||
        !std::isfinite(m.alpha) || (m.kind == MRS_GGX && !(m.alpha > 0.0f && m.alpha <= 1.0f)))
      return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: invalid material " + std::to_string(i));
  }
  for (int i = 0; i < n; ++i) {
    if (d->tri_material[i] >= (uint32_t)d->num_materials)
      return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: material index out of range at triangle " + std::to_string(i));
    const float* v = d->vertices + 9 * (size_t)i;
    if (!finite3(v) || !finite3(v + 3) || !finite3(v + 6))
      return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: non-finite vertex at triangle " + std::to_string(i));
  }
  for (int i = 0; i < d->num_lights; ++i) {
    const mrs_quad_light& l = d->lights[i];
    if (l.tri[0] < 0 || l.tri[0] >= n || l.tri[1] < 0 || l.tri[1] >= n)
      return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: light triangle index out of range");
    if (!finite3(l.corner) || !finite3(l.edge_u) || !finite3(l.edge_v) || !finite3(l.emission) ||
        len(crs(d3(l.edge_u), d3(l.edge_v))) <= 0.0)
      return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: degenerate light " + std::to_string(i));
  }
  const mrs_camera& c = d->camera;
  if (!finite3(c.pos) || !finite3(c.look_at) || !finite3(c.up) || !(c.vfov_deg > 0.0f && c.vfov_deg < 180.0f))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: invalid camera");
  D3 f = sub(d3(c.look_at), d3(c.pos));
  if (len(f) <= 0.0 || len(crs(nrm(f), d3(c.up))) <= 1e-9)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_create: camera up is parallel to the view direction");
  mrs_scene* s = new mrs_scene();
  mrs_status rc = scene_create_impl(d, s);
  if (rc != MRS_OK) {
    free_scene(s);
    delete s;
    return rc;
  }
  *out = s;
  return MRS_OK;
}

mrs_status mrs_scene_destroy(mrs_scene* s) {
  if (!s) return MRS_OK;
  (void)hipDeviceSynchronize();
  free_scene(s);
  delete s;
  return MRS_OK;
}

mrs_status mrs_build_bvh(mrs_scene* s) {
  if (!s) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_build_bvh: scene is NULL");
  if (s->bvh_built) return MRS_OK;
  mrs_tuning t;
  get_tuning(&t);
  mrs_status rc = lbvh_build(s, current_stream(), t.bvh_leaf_max, t.bvh_builder);
  if (rc != MRS_OK) return rc;
  s->view.root = s->root4;
  s->view.nodes = s->d_nodes4;
  s->view.nodes_q = s->d_nodes4q;
  s->view.nnodes = s->count4;
  return MRS_OK;
}

void mrs_render_opts_default(mrs_render_opts* o) {
  if (!o) return;
  o->rr_start = 3;
  o->x0 = o->y0 = 0;
  o->win_w = o->win_h = 0;
  o->accum_fp64 = -1;
  o->mis = 0;
  o->lens_radius = 0.0f;
  o->focus_dist = 0.0f;
  o->cam_motion[0] = o->cam_motion[1] = o->cam_motion[2] = 0.0f;
  o->out_sumsq_dev = nullptr;
  o->out_layers_dev = nullptr;
}

namespace {
mrs_status validate_render(const char* fn, const mrs_scene* s, int32_t W, int32_t H, int32_t spp,
                           int32_t max_depth, uint64_t seed, const mrs_render_opts* opts,
                           float* out_rgb, float* out_aux, RenderArgs* a) {
  const std::string f(fn);
  mrs_render_opts o;
  mrs_render_opts_default(&o);
  if (opts) o = *opts;
  if (o.rr_start < 0) return fail(MRS_ERR_INVALID_ARGUMENT, f + ": rr_start < 0");
  if (o.mis != 0 && o.mis != 1) return fail(MRS_ERR_INVALID_ARGUMENT, f + ": mis must be 0 or 1");
  if (!(o.lens_radius >= 0.0f) || !std::isfinite(o.lens_radius) ||
      (o.lens_radius > 0.0f && !(o.focus_dist > 0.0f && std::isfinite(o.focus_dist))))
    return fail(MRS_ERR_INVALID_ARGUMENT,
                f + ": lens_radius must be >= 0, with a positive finite focus_dist");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(o.cam_motion[k]))
      return fail(MRS_ERR_INVALID_ARGUMENT, f + ": cam_motion must be finite");
  if (!s) return fail(MRS_ERR_INVALID_ARGUMENT, f + ": scene is NULL");
  if (W < 1 || H < 1 || W > 16384 || H > 16384)
    return fail(MRS_ERR_INVALID_ARGUMENT, f + ": W and H must be in [1, 16384]");
  if (spp < 1 || spp > (1 << 20))
    return fail(MRS_ERR_INVALID_ARGUMENT, f + ": spp must be in [1, 2^20]");
  if (max_depth < 0 || max_depth > 64)
    return fail(MRS_ERR_INVALID_ARGUMENT, f + ": max_depth must be in [0, 64]");

  const int ww = o.win_w ? o.win_w : W, wh = o.win_h ? o.win_h : H;
  if (o.x0 < 0 || o.y0 < 0 || ww < 1 || wh < 1 || o.x0 + ww > W || o.y0 + wh > H)
    return fail(MRS_ERR_INVALID_ARGUMENT, f + ": window outside the image");
  if (!out_rgb) return fail(MRS_ERR_INVALID_ARGUMENT, f + ": out_rgb is NULL");
  if (((uintptr_t)out_rgb | (uintptr_t)out_aux | (uintptr_t)o.out_sumsq_dev |
       (uintptr_t)o.out_layers_dev) & 3u)
    return fail(MRS_ERR_INVALID_ARGUMENT, f + ": outputs must be 4-byte aligned");
  if (!s->bvh_built) return fail(MRS_ERR_NOT_READY, f + ": call mrs_build_bvh first");
  a->W = W;
  a->H = H;
  a->spp = spp;
  a->max_depth = max_depth;
  a->rr_start = o.rr_start;
  a->seed = seed;
  a->x0 = o.x0;
  a->y0 = o.y0;
  a->ww = ww;
  a->wh = wh;
  a->fp64 = o.accum_fp64 < 0 ? spp >= 1024 : o.accum_fp64 != 0;
  a->mis = o.mis != 0;
  a->lens_r = o.lens_radius;
  a->focus = o.focus_dist;
  for (int k = 0; k < 3; ++k) a->motion[k] = o.cam_motion[k];
  a->out_rgb = out_rgb;
  a->out_aux = out_aux;
  a->out_sumsq = o.out_sumsq_dev;
  a->out_layers = o.out_layers_dev;
  return MRS_OK;
}
}  // namespace

mrs_status mrs_render_ex(const mrs_scene* s, int32_t W, int32_t H, int32_t spp, int32_t max_depth,
                         uint64_t seed, const mrs_render_opts* opts, float* out_rgb,
                         float* out_aux) {
  RenderArgs a;
  mrs_status rc = validate_render("mrs_render", s, W, H, spp, max_depth, seed, opts, out_rgb,
                                  out_aux, &a);
  if (rc != MRS_OK) return rc;
  return render(s, a, current_stream());
}

mrs_status mrs_render_ex_noalloc(const mrs_scene* s, int32_t W, int32_t H, int32_t spp,
                                 int32_t max_depth, uint64_t seed, const mrs_render_opts* opts,
                                 float* out_rgb, float* out_aux) {
  RenderArgs a;
  mrs_status rc = validate_render("mrs_render_ex_noalloc", s, W, H, spp, max_depth, seed, opts,
                                  out_rgb, out_aux, &a);
  if (rc != MRS_OK) return rc;
  return render_noalloc(s, a, current_stream());
}

mrs_status mrs_batch_create(const mrs_job* jobs, int32_t n, mrs_batch** out) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_create: out is NULL");
  *out = nullptr;
  if (!jobs || n < 1 || n > MAX_JOBS)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_create: need 1..255 jobs");
  std::vector<DevJob> dj;
  for (int i = 0; i < n; ++i) {
    const mrs_job& j = jobs[i];
    RenderArgs a;
    mrs_status rc = validate_render(("mrs_batch_create: job " + std::to_string(i)).c_str(),
                                    j.scene, j.W, j.H, j.spp, j.max_depth, j.seed, &j.opts,
                                    j.out_rgb_dev, j.out_aux_dev, &a);
    if (rc != MRS_OK) return rc;
    dj.push_back(make_job(j.scene, a));
  }
  return batch_create(dj, out);
}

mrs_status mrs_batch_render(mrs_batch* b) {
  if (!b) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_render: batch is NULL");
  return batch_render(b, current_stream());
}

mrs_status mrs_batch_render_begin(mrs_batch* b) {
  if (!b) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_render_begin: batch is NULL");
  return batch_render_begin(b, current_stream());
}

mrs_status mrs_batch_render_fork(mrs_batch* b) {
  if (!b) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_render_fork: batch is NULL");
  return batch_render_fork(b, current_stream());
}

mrs_status mrs_batch_render_end(mrs_batch* b) {
  if (!b) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_render_end: batch is NULL");
  return batch_render_end(b, current_stream());
}

mrs_status mrs_batch_set_seeds(mrs_batch* b, const uint64_t* seeds) {
  if (!b || !seeds) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_batch_set_seeds: NULL argument");
  return batch_set_seeds(b, seeds, current_stream());
}

mrs_status mrs_batch_destroy(mrs_batch* b) {
  batch_destroy(b);
  return MRS_OK;
}

mrs_status mrs_release_workspaces(void) {
  release_workspaces();
  return MRS_OK;
}

mrs_status mrs_render(const mrs_scene* s, int32_t W, int32_t H, int32_t spp, int32_t max_depth,
                      uint64_t seed, float* out_rgb, float* out_aux) {
  return mrs_render_ex(s, W, H, spp, max_depth, seed, nullptr, out_rgb, out_aux);
}

mrs_status mrs_get_counters(int64_t out[MRS_NUM_COUNTERS], int32_t reset) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_get_counters: out is NULL");
  return get_counters(out, reset != 0, current_stream());
}

mrs_status mrs_image_metrics(const float* img, const float* ref, int64_t count, double lambda1,
                             double lambda2, double out[3]) {
  if (!img || !ref || !out || count <= 0)
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_image_metrics: bad arguments");
  if (!(lambda2 > 0.0)) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_image_metrics: lambda2 <= 0");
  static double* d_out = nullptr;
  if (!d_out) MRS_TRY_HIP(hipMalloc(&d_out, sizeof(double) * 2));
  hipStream_t st = current_stream();
  mrs_status rc = image_metrics(img, ref, count, lambda1, lambda2, d_out, st);
  if (rc != MRS_OK) return rc;
  double h[2];
  MRS_TRY_HIP(hipMemcpyAsync(h, d_out, sizeof h, hipMemcpyDeviceToHost, st));
  MRS_TRY_HIP(hipStreamSynchronize(st));
  out[0] = h[0];
  out[1] = h[0] > 0.0 ? 10.0 * std::log10(1.0 / h[0]) : INFINITY;
  out[2] = h[1];
  return MRS_OK;
}

mrs_status mrs_set_count_work(int32_t on) {
  set_count_work(on != 0);
  return MRS_OK;
}

mrs_status mrs_profile_enable(int32_t on) { return prof_enable(on != 0); }
mrs_status mrs_profile_select(uint32_t mask) { return prof_select(mask); }

mrs_status mrs_profile_read(double* ms, int64_t* launches) {
  if (!ms || !launches) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_profile_read: NULL output");
  return prof_read(ms, launches);
}

mrs_status mrs_get_tuning(mrs_tuning* out) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_get_tuning: out is NULL");
  get_tuning(out);
  return MRS_OK;
}

mrs_status mrs_set_tuning(const mrs_tuning* t) {
  if (!t) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_set_tuning: NULL");
  return set_tuning(t);
}

mrs_status mrs_debug_conv_launches(int64_t* out, int32_t reset) {
  if (!out) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_conv_launches: out is NULL");
  conv_launch_counts(out, reset != 0);
  return MRS_OK;
}

mrs_status mrs_debug_philox(int32_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  if (n < 0 || (n > 0 && (!ctr || !key || !out)))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_philox: bad arguments");
  return debug_philox(n, ctr, key, out, current_stream());
}

mrs_status mrs_debug_closest_hit(const mrs_scene* s, int32_t n, const float* o, const float* d,
                                 const int32_t* skip, float* t, int32_t* prim, float* b) {
  if (!s || n < 0 || (n > 0 && (!o || !d || !t || !prim || !b)))
    return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_closest_hit: bad arguments");
  if (!s->bvh_built) return fail(MRS_ERR_NOT_READY, "mrs_debug_closest_hit: BVH not built");
  return debug_closest_hit(s, n, o, d, skip, t, prim, b, current_stream());
}

mrs_status mrs_debug_bvh(const mrs_scene* s, float* nodes, int32_t* leaf_prim, uint32_t* morton,
                         int32_t* root_ref) {
  if (!s) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_bvh: scene is NULL");
  if (!s->bvh_built) return fail(MRS_ERR_NOT_READY, "mrs_debug_bvh: BVH not built");
  MRS_TRY_HIP(hipStreamSynchronize(current_stream()));
  const int n = s->ntris;
  if (nodes && n >= 2) MRS_TRY_HIP(hipMemcpy(nodes, s->d_nodes, sizeof(float4) * 4 * (size_t)(n - 1), hipMemcpyDeviceToHost));
  if (leaf_prim && n > 0) MRS_TRY_HIP(hipMemcpy(leaf_prim, s->d_leaf_prim, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
  if (morton && n > 0) MRS_TRY_HIP(hipMemcpy(morton, s->d_morton, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
  if (root_ref) *root_ref = (int32_t)s->root;
  return MRS_OK;
}

mrs_status mrs_scene_bvh_builder(const mrs_scene* s, int32_t* builder) {
  if (!s || !builder) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_scene_bvh_builder: NULL argument");
  if (!s->bvh_built) return fail(MRS_ERR_NOT_READY, "mrs_scene_bvh_builder: BVH not built");
  *builder = s->builder;
  return MRS_OK;
}

mrs_status mrs_debug_bvh4(const mrs_scene* s, float* nodes, int32_t* count, uint32_t* root_ref,
                          int32_t* leaf_max) {
  if (!s) return fail(MRS_ERR_INVALID_ARGUMENT, "mrs_debug_bvh4: scene is NULL");
  if (!s->bvh_built) return fail(MRS_ERR_NOT_READY, "mrs_debug_bvh4: BVH not built");
  MRS_TRY_HIP(hipStreamSynchronize(current_stream()));
  if (nodes && s->count4 > 0)
    MRS_TRY_HIP(hipMemcpy(nodes, s->d_nodes4, sizeof(float4) * 8 * (size_t)s->count4,
                          hipMemcpyDeviceToHost));
  if (count) *count = (int32_t)s->count4;
  if (root_ref) *root_ref = s->root4;
  if (leaf_max) *leaf_max = s->leaf_max;
  return MRS_OK;
}

}  // extern "C"
