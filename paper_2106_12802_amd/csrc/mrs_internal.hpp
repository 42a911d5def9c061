// Internal declarations shared by the libmrs translation units (GPU side only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "mrs.h"

namespace mrs {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
mrs_status fail(mrs_status st, const std::string& msg);
mrs_status check_hip(hipError_t e, const char* what);
hipStream_t current_stream();
void set_stream(hipStream_t s);
const std::string& t_error_ref();

#define MRS_TRY_HIP(expr)                                       \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) return ::mrs::check_hip(e_, #expr);   \
  } while (0)

#define MRS_TRY_STATUS(expr)          \
  do {                                \
    mrs_status s_ = (expr);           \
    if (s_ != MRS_OK) return s_;      \
  } while (0)

// ------------------------------------------------------------------ device scene
constexpr uint32_t LEAF_BIT = 0x80000000u;
constexpr uint32_t NO_PRIM = 0xffffffffu;
constexpr int MAX_LIGHTS = 255;
constexpr int MAX_STACK = 64;  // Karras trees over unique 64-bit keys are <= 64 deep

// Four-wide BVH collapsed from the binary LBVH (128 B per node, one cache
// line): child boxes as structure-of-arrays float4s (lo.x, lo.y, lo.z, hi.x,
// hi.y, hi.z of children 0..3), then the 4 child references and 4 pad words.
// Reference: EMPTY4 (no child), LEAF_BIT | (count - 1) << 24 | first (leaf
// records first .. first + count - 1, count <= 4), or a node index.
constexpr uint32_t EMPTY4 = 0xffffffffu;
constexpr int LEAF4_MAX = 4;
__host__ __device__ constexpr uint32_t leaf4_ref(uint32_t first, uint32_t count) {
  return LEAF_BIT | ((count - 1u) << 24) | first;
}

struct DevMaterial {  // 32 B, read through the scalar/vector caches
  float4 color_alpha; // rgb = albedo or F0, w = GGX roughness
  float4 emis_kind;   // rgb = emission, w = kind (as float: 0, 1, 2)
};

struct DevLight {  // 80 B
  float4 corner;   // xyz
  float4 eu;       // xyz
  float4 ev;       // xyz
  float4 le;       // rgb emission
  float4 normal;   // xyz unit normal, w = area
  int32_t tri0, tri1, pad0, pad1;
};

struct SceneView {  // passed by value to kernels
  int32_t ntris;
  int32_t nlights;
  uint32_t root;           // BVH4 reference of the root
  uint32_t nnodes;         // BVH4 nodes
  const float4* nodes;     // nnodes * 8 float4 (BVH4)
  const float4* nodes_q;   // nnodes * 4 float4 (BVH4, quantized child boxes)
  const float4* leaf_tri;  // ntris*3 float4: (v0, prim bits) (e1, -) (e2, -) in leaf order
  const float4* prim_ng;   // ntris: unit geometric normal, w = bits(material | flags)
  const float4* prim_n;    // ntris*3: per-corner shading normals (smooth triangles)
  const DevMaterial* mats;
  const DevLight* lights;
  float env_r, env_g, env_b;
  // camera basis (computed in FP64 on the host, rounded once)
  float cam_px, cam_py, cam_pz;
  float cam_fx, cam_fy, cam_fz;
  float cam_rx, cam_ry, cam_rz;
  float cam_vx, cam_vy, cam_vz;
  float cam_tan_half;
};

// One render of a batch: its scene, image, window, sampling and outputs.
// Paths of all jobs form one index space: job j owns [first, first + spp * npix)
// pixel-major (each pixel's samples consecutive); pix_first indexes its pixels in the concatenated
// pixel space; acc_off locates its accumulators (bytes).
struct DevJob {
  SceneView sv;
  int32_t W, H, x0, y0, ww, wh;
  int32_t spp, max_depth, rr_start, fp64;
  int32_t mis, moving;
  float lens_r, focus, motion_x, motion_y, motion_z, pad0;
  // path order of the full 8-pixel tile rows: row position p holds tile row
  // (p * row_mul) mod rows_full (row_inv is row_mul's inverse mod rows_full)
  uint32_t rows_full, row_mul, row_inv, pad1;
  uint32_t seed_lo, seed_hi;
  int64_t first, pix_first, acc_off;
  float* out_rgb;
  float* out_aux;
  float* out_sq;
  float* out_layers;  // 9 per pixel: emission, diffuse, glossy (or null)
};

constexpr int MAX_JOBS = 255;                // job ids travel in 8 bits
constexpr int32_t MAX_TRIS = (1 << 24) - 2;  // primitive ids travel in 24 bits

// prim_ng.w packs: bits 0..23 material index, bit 24 smooth, bit 25 listed light
constexpr uint32_t PRIM_SMOOTH = 1u << 24;
constexpr uint32_t PRIM_LISTED = 1u << 25;
constexpr uint32_t PRIM_MAT_MASK = 0x00ffffffu;

}  // namespace mrs

struct mrs_scene {
  int32_t ntris = 0;
  int32_t nmats = 0;
  int32_t nlights = 0;
  bool bvh_built = false;
  // device buffers
  float4* d_tri_src = nullptr;  // ntris*3: v0, v1, v2 in primitive order (w unused)
  float4* d_prim_ng = nullptr;
  float4* d_prim_n = nullptr;
  float4* d_leaf_tri = nullptr;
  float4* d_nodes = nullptr;   // binary LBVH: (ntris-1) * 4 float4
  float4* d_nodes4 = nullptr;  // BVH4: count4 * 8 float4
  float4* d_nodes4q = nullptr; // the same nodes quantized: count4 * 4 float4
  uint32_t count4 = 0;
  uint32_t root4 = 0;
  int32_t leaf_max = mrs::LEAF4_MAX;  // triangles per BVH4 leaf the build may group
  int32_t builder = MRS_BVH_LBVH;     // the builder that made the binary tree
  uint32_t* d_morton = nullptr;     // Morton codes in leaf order
  uint32_t* d_leaf_prim = nullptr;  // primitive ids in leaf order
  mrs::DevMaterial* d_mats = nullptr;
  mrs::DevLight* d_lights = nullptr;
  mrs::SceneView view{};
  uint32_t root = 0;
};

namespace mrs {
// lbvh.hip
mrs_status lbvh_build(mrs_scene* s, hipStream_t st, int leaf_max, int builder);
// trace.hip
struct RenderArgs {
  int32_t W, H, spp, max_depth, rr_start;
  uint64_t seed;
  int32_t x0, y0, ww, wh;
  bool fp64;
  bool mis;
  float lens_r, focus, motion[3];
  float* out_rgb;
  float* out_aux;
  float* out_sumsq;
  float* out_layers;
};
mrs_status render(const mrs_scene* s, const RenderArgs& a, hipStream_t st);
// The same render with its workspace in a fixed device array (no allocation).
mrs_status render_noalloc(const mrs_scene* s, const RenderArgs& a, hipStream_t st);
DevJob make_job(const mrs_scene* s, const RenderArgs& a);
// a batch of validated jobs: job table, accumulators and its own workspace
mrs_status batch_create(const std::vector<DevJob>& jobs, mrs_batch** out);
mrs_status batch_render(mrs_batch* b, hipStream_t st);
mrs_status batch_render_begin(mrs_batch* b, hipStream_t st);
mrs_status batch_render_end(mrs_batch* b, hipStream_t st);
mrs_status batch_render_fork(mrs_batch* b, hipStream_t st);
mrs_status batch_set_seeds(mrs_batch* b, const uint64_t* seeds, hipStream_t st);
void batch_destroy(mrs_batch* b);
// frees the per-stream workspaces (synchronises the device)
void release_workspaces();
mrs_status debug_closest_hit(const mrs_scene* s, int32_t n, const float* o, const float* d,
                             const int32_t* skip, float* t, int32_t* prim, float* b,
                             hipStream_t st);
mrs_status debug_philox(int32_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                        hipStream_t st);
mrs_status get_counters(int64_t* out, bool reset, hipStream_t st);
void get_tuning(mrs_tuning* t);
mrs_status set_tuning(const mrs_tuning* t);
int conv_small_tiles();  // mrs_tuning.conv_small_tiles in force
int net_fused_blocks();  // mrs_tuning.net_fused_blocks in force
// Launches of each network conv kernel instance since the last reset (host
// counters, in the order of mrs_debug_conv_launches).
void conv_launch_counts(int64_t* out, bool reset);
void set_count_work(bool on);
// metrics.hip: out_dev[0] = sRGB MSE, out_dev[1] = RelMSE (FP64, device)
mrs_status image_metrics(const float* img, const float* ref, int64_t n, double lam1, double lam2,
                         double* out_dev, hipStream_t st);
// prof.hip: HIP-event timing of kernel launches by id
enum KernelId {
  KID_GENERATE = 0,
  KID_EXTEND = 1,
  KID_SHADE = 2,
  KID_SHADOW = 3,
  KID_ACCUMULATE = 4,
  KID_RESOLVE = 5,
  KID_CNN_PREP = 6,
  KID_CNN_HR = 7,
  KID_CNN_LR = 8,
  KID_CNN_REC = 9,
  KID_TRAIN_FWD = 10,
  KID_TRAIN_BWD = 11,
  KID_TRAIN_ADAM = 12,
  KID_TAIL = 13,
};
// While a ProfPause is alive on a thread, its launches record no timing events.
struct ProfPause {
  ProfPause();
  ~ProfPause();
  ProfPause(const ProfPause&) = delete;
  ProfPause& operator=(const ProfPause&) = delete;
};
void prof_begin(int id, hipStream_t st);
void prof_end(int id, hipStream_t st);
mrs_status prof_enable(bool on);
mrs_status prof_select(uint32_t mask);
mrs_status prof_read(double* ms, int64_t* launches);
}  // namespace mrs
