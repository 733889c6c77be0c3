// Host implementation of the C ABI in include/xpbd.h: problem validation,
// device layout, the frame / substep / iteration / set loops that launch the
// forward and reverse kernels, per-frame checkpoints and the record of
// projection inputs replayed by the adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/xpbd.h"
#include "xpbd_kernels.hpp"
#include "xpbd_pack_kernels.hpp"

using namespace xpbd;

namespace {

struct Fail {
  xpbd_status st;
  std::string msg;
};

[[noreturn]] void fail(xpbd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Fail{st, buf};
}

#define HIPCHK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) fail(XPBD_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

inline unsigned nblocks(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// Host-side roctx range over a scope (frames, substeps, Gauss-Seidel sweeps):
// what rocprofv3 --marker-trace shows of the library's launch loops; a call
// costs a few tens of nanoseconds when no tool listens.
struct Range {
  explicit Range(const char* m) { roctxRangePushA(m); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct SetInfo {
  int type;
  int begin;   // first internal record of this set within its type's arrays
  int count;
  size_t tape_off;   // byte offset of this set's record inside one iteration
};

// bytes of the per-projection record per item, by type (scaled by sizeof T / 4)
// timed kernel families: 2 type (+1 reverse) for types 0..3 (6/7: sphere and
// body contact), 8/9 persistent frame, 10/11 LDS group, 12/13 membrane sets
constexpr int kProfFamilies = 14;
inline int prof_family(int type, bool rev) {
  return (type == XPBD_TRI ? 12 : type == XPBD_BODY ? 6 : 2 * type) + (rev ? 1 : 0);
}

inline size_t tape_item_bytes(int type, size_t tsz) {
  switch (type) {
    case XPBD_DIST: return 4 * tsz;
    case XPBD_BEND: return 10 * tsz;
    case XPBD_TET: return 12 * tsz;
    case XPBD_TRI: return 12 * tsz;
    default: return 4 * tsz;
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

}  // namespace

// Partial sums of the goal reduction for xpbd_goal_weighted_noalloc: a
// file-scope device array (one copy per GPU, held until the process ends)
// instead of memory the context allocates.  On the host `scratch` names a
// stand-in, not a device address: kernels get the address that
// hipGetSymbolAddress returned for the device, kept in g_scratch_addr.
constexpr size_t kGoalScratchDoubles = (size_t)1 << 21;   // 16 MiB
static __device__ __align__(256) double scratch[kGoalScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};
}  // namespace

struct xpbd_ctx_s {
  std::string err;
  int device = 0;   // the GPU the context was created on
  xpbd_dtype dtype;
  size_t tsz;
  int V = 0, n_dist = 0, n_bend = 0, n_tet = 0, n_contact = 0, n_tri = 0;
  // body collider: mesh, contact items, pairing per substep, pairing grid
  int body_nv = 0, body_nt = 0, n_bc = 0;
  double b_tau = 0, b_alpha = 0, b_radius = 0;
  int4* body_tris = nullptr;
  int* bc_vid = nullptr; void* bc_lam = nullptr; void* bc_lamb = nullptr;
  int* body_pair = nullptr; size_t body_pair_cap = 0;   // [F * S][n_bc]
  int* grid_off = nullptr; size_t grid_off_cap = 0; int* grid_tris = nullptr; size_t grid_tris_cap = 0;
  BodyGrid grid{};
  std::vector<int> body_tris_h;     // host copy [body_nt][3]
  const void* cur_body_x = nullptr;
  double dt, h;
  int S, K;
  double g[3];
  size_t budget;
  int gamma_one;
  int tape_mode_opt;
  int block = kBlock;   // workgroup size of the per-set kernels
  bool group_stream = false;   // LDS groups: records streamed from the global image
  int record_kind = 0;         // 0 record of every projection's inputs, 1 snapshots of each group launch
  bool want_ab = true;         // this adjoint asks for distance or bending compliance gradients
  char* scratch = nullptr;     // record_kind 1, entries streamed: one group launch's replayed record
  size_t scratch_bytes = 0;
  int group_block = kBlock;    // workgroup size of the LDS group kernels
  int tape_mode_used = 0;
  double tau = 0, alpha_c = 0;
  std::vector<SetInfo> sets;
  size_t iter_tape_bytes = 0;
  int64_t proj_per_iter = 0;

  // device memory registry
  std::vector<DevBuf> bufs;
  size_t dev_bytes = 0;

  // persistent records (internal order)
  int2* dist_idx = nullptr; void* dist_rest = nullptr; int* dist_perm = nullptr;
  int4* bend_idx = nullptr; void* bend_theta0 = nullptr; int* bend_perm = nullptr;
  int4* tet_idx = nullptr; void* tet_B = nullptr; int* tet_perm = nullptr; double* tet_nu = nullptr;
  double* tet_vol = nullptr;
  // tet parameter index per tet (internal order): the caller's tet index, or
  // its material; material clusters also keep each material's tets
  // (internal indices, ascending) as mat_items[mat_off[m] .. mat_off[m+1])
  int* tet_pidx = nullptr;
  int n_mat = 0;
  int* mat_off = nullptr; int* mat_items = nullptr;
  // membrane triangles: corners, Dm^-1 [4][n], material-space area
  int4* tri_idx = nullptr; void* tri_B = nullptr; int* tri_perm = nullptr; double* tri_area = nullptr;
  int* contact_vid = nullptr;
  int* contact_order = nullptr;   // per contact set: set-local items by ascending vertex
  void* w = nullptr;              // [V] inverse mass (T)
  // two device copies of the per-set kernels' parameter block (kDevBlk bytes
  // each): [0] written and read by forward substeps, [1] by reverse substeps,
  // so the adjoint's recompute stream and reverse stream never share one
  void* dev_blk = nullptr;
  // per forward
  void* dist_at = nullptr; void* bend_at = nullptr;
  void* tet_atD = nullptr; void* tet_atH = nullptr; void* tet_gamma = nullptr;
  void* dist_lam = nullptr; void* bend_lam = nullptr; void* tet_lamD = nullptr; void* tet_lamH = nullptr;
  void* contact_lam = nullptr;
  void* tri_at = nullptr; void* tri_lam = nullptr;   // [4][n], [3][n]
  void* X = nullptr; void* Vv = nullptr; void* Xp = nullptr;
  int* flag = nullptr;
  double* parts = nullptr; size_t parts_n = 0;
  // checkpoints
  void* ckX = nullptr; void* ckV = nullptr; int ck_frames = 0;
  // adjoint
  void* XB = nullptr; void* VB = nullptr;
  void* dist_lamb = nullptr; void* dist_ab = nullptr; double* dist_acc = nullptr;
  void* bend_lamb = nullptr; void* bend_ab = nullptr; double* bend_acc = nullptr;
  void* tet_lambD = nullptr; void* tet_lambH = nullptr; void* tet_eb = nullptr; double* tet_acc = nullptr;
  void* contact_lamb = nullptr; void* contact_sacc = nullptr;
  void* tri_lamb = nullptr; void* tri_ab = nullptr; double* tri_acc = nullptr;   // [3][n], [4][n], [4][n]
  void* tape = nullptr; size_t tape_cap = 0;

  // LDS groups
  struct Group {
    int a, b;                 // sets [a, b)
    bool lds = false;         // run as one launch per iteration
    int P = 0;
    size_t smem_fwd = 0, smem_rev = 0;   // vertex tile + constant entries + state (+ record of inputs)
    size_t smem_tile = 0;                 // vertex tile only (entries and state streamed)
    int64_t items = 0;        // projections per iteration inside the group
    bool heavy = false;       // has tet or membrane sets (kernels with those projections)
    int* pv_start = nullptr; int* pv = nullptr; int* cnt = nullptr; int* set_type = nullptr;
    long long* img = nullptr; long long* fmul = nullptr; long long* rmul = nullptr;   // per patch offsets
    long long* tpos = nullptr; int* rec_first = nullptr;
    long long tape_off = 0;   // inside one iteration's record
    size_t tape_bytes = 0;
    // snapshot records (record_kind 1): staged vertices, forward state image
    // bytes and its first offset, positions / multipliers inside one iteration
    size_t n_staged = 0, fmul_bytes = 0;
    long long fmul_lo = 0, snap_x_off = 0, snap_l_off = 0;
    size_t max_tbytes = 0;     // largest patch record of one iteration
    bool replay_lds = false;   // entries streamed: the replayed record fits in LDS beside the two tiles
  };
  std::vector<Group> groups;
  std::vector<int> group_at_start, group_at_end;   // per set: group starting / ending there, -1 none
  char* gimg = nullptr;                                 // group constant entries
  char* gfmul = nullptr; char* grmul = nullptr;         // group forward multipliers, reverse state
  long long* gpos[4] = {nullptr, nullptr, nullptr, nullptr};   // dist / bend / tet / membrane: entry offset in gimg, -1 none
  size_t lds_limit = 65536;
  int max_group_lds = 0;

  // persistent program launches
  bool persistent = false;
  int prog_blocks_opt = 0;
  int prog_grid = 0;
  Phase* fw_prog = nullptr; Phase* rv_prog = nullptr;
  int n_fw_prog = 0, n_rv_prog = 0;
  unsigned* bar = nullptr;
  int* abort_flag = nullptr;

  // packs: the context serves at most one job at a time
  bool in_pack = false;
  uint8_t* pack_mask = nullptr;   // device [F] goal frames of the current job
  int pack_mask_cap = 0;
  hipEvent_t pack_event = nullptr;  // recorded after the last work of its latest job

  // implicit adjoint work space (substep end states, CG vectors)
  void* imp_buf = nullptr;
  size_t imp_cap = 0;

  // forward bookkeeping for the adjoint
  bool have_forward = false;
  bool fwd_recorded = false;
  int fwd_rec_from = 0;          // first frame whose record the forward kept (frames >= it)
  int record_frames_opt = 0;     // tape_mode 4: most final frames the forward records (0 = all that fit)
  // adjoint: while one library stream reverses a frame, another recomputes
  // an earlier frame's record (events order the two); serial_adjoint = 1
  // runs every step on the call's stream
  int serial_adjoint = 0;
  hipStream_t adj_rec = nullptr, adj_rev = nullptr;
  int adj_streams_used = 0;   // streams the last adjoint ran on (1 or 2)
  std::vector<hipEvent_t> adj_events;
  int fwd_frames = 0;
  xpbd_params fwd_params{};

  // profiling
  int prof_stride = 0;
  int64_t prof_counter = 0;
  struct Ev { hipEvent_t a, b; int fam; int64_t items; };
  std::vector<Ev> ev_pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
  int64_t prof_launch[kProfFamilies] = {0};
  double prof_ms[kProfFamilies] = {0};
  int64_t prof_items[kProfFamilies] = {0};

  ~xpbd_ctx_s() {
    for (hipStream_t* s : {&adj_rec, &adj_rev})
      if (*s) {
        (void)hipStreamSynchronize(*s);
        (void)hipStreamDestroy(*s);
      }
    for (hipEvent_t e : adj_events) (void)hipEventDestroy(e);
    if (pack_event) {
      (void)hipEventSynchronize(pack_event);
      (void)hipEventDestroy(pack_event);
    }
    for (auto& b : bufs) if (b.p) (void)hipFree(b.p);
    for (auto& e : ev_pending) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto& e : ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  }

  void* alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    size_t b = align256(bytes);
    if (budget && dev_bytes + b > budget)
      fail(XPBD_ERR_OOM, "device memory budget of %zu bytes exceeded (%zu in use, %zu requested)", budget,
           dev_bytes, b);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(XPBD_ERR_OOM, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
    }
    bufs.push_back({p, b});
    dev_bytes += b;
    return p;
  }
  void release(void*& p) {
    if (!p) return;
    for (auto it = bufs.begin(); it != bufs.end(); ++it)
      if (it->p == p) {
        (void)hipFree(p);
        dev_bytes -= it->n;
        bufs.erase(it);
        break;
      }
    p = nullptr;
  }
  template <class U> void upload(void* dst, const std::vector<U>& v) {
    if (!v.empty()) HIPCHK(hipMemcpy(dst, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice));
  }
};

namespace {

// ===================================================================== rest data (host, FP64)

struct H3 { double x, y, z; };
inline H3 hsub(H3 a, H3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double hdot(H3 a, H3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline H3 hcross(H3 a, H3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline H3 hv(const double* p, int k) { return {p[3 * k], p[3 * k + 1], p[3 * k + 2]}; }

// signed dihedral angle of hinge (p0, p1) with wings p2, p3; false if degenerate
bool rest_dihedral(H3 p0, H3 p1, H3 p2, H3 p3, double* th) {
  H3 e = hsub(p1, p0), a = hsub(p2, p0), b = hsub(p3, p0);
  H3 n1 = hcross(e, a), n2 = hcross(b, e);
  double le2 = hdot(e, e);
  if (!(le2 > 0) || !(hdot(n1, n1) > 0) || !(hdot(n2, n2) > 0)) return false;
  *th = std::atan2(hdot(hcross(n1, n2), e) / std::sqrt(le2), hdot(n1, n2));
  return true;
}

// Dm^-1 (row-major) and rest volume; false if det <= 0
bool rest_tet(H3 p0, H3 p1, H3 p2, H3 p3, double B[9], double* vol) {
  H3 c0 = hsub(p1, p0), c1 = hsub(p2, p0), c2 = hsub(p3, p0);
  // Dm = [c0 c1 c2]; det = c0 . (c1 x c2); inverse rows = (c1 x c2, c2 x c0, c0 x c1) / det
  H3 r0 = hcross(c1, c2), r1 = hcross(c2, c0), r2 = hcross(c0, c1);
  double det = hdot(c0, r0);
  if (!(det > 0)) return false;
  const H3 rows[3] = {r0, r1, r2};
  for (int r = 0; r < 3; ++r) {
    B[3 * r + 0] = rows[r].x / det;
    B[3 * r + 1] = rows[r].y / det;
    B[3 * r + 2] = rows[r].z / det;
  }
  *vol = det / 6.0;
  return true;
}

template <class T> std::vector<T> cast_vec(const std::vector<double>& v) {
  std::vector<T> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
  return o;
}

// ===================================================================== profiling

void prof_begin(xpbd_ctx c, hipStream_t st, int fam, int64_t items, xpbd_ctx_s::Ev* out, bool* on) {
  *on = false;
  if (!c->prof_stride) return;
  // sample one launch in prof_stride, chosen by a hash of the launch count
  // rather than every n-th, so launch sequences whose period shares a factor
  // with the stride (e.g. 21 sets per iteration, stride 7) are not aliased
  const uint64_t k = (uint64_t)(c->prof_counter++) * 0x9E3779B97F4A7C15ull;
  if (((k >> 32) % (uint64_t)c->prof_stride) != 0) return;
  hipEvent_t a, b;
  if (!c->ev_free.empty()) {
    a = c->ev_free.back().first;
    b = c->ev_free.back().second;
    c->ev_free.pop_back();
  } else {
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
  }
  HIPCHK(hipEventRecord(a, st));
  *out = {a, b, fam, items};
  *on = true;
}
void prof_end(xpbd_ctx c, hipStream_t st, xpbd_ctx_s::Ev& e, bool on) {
  if (!on) return;
  HIPCHK(hipEventRecord(e.b, st));
  c->ev_pending.push_back(e);
}

// ===================================================================== launches

// body pairing of every substep of an F-frame rollout
void ensure_body_pairs(xpbd_ctx c, int F) {
  if (!c->n_bc) return;
  size_t need = (size_t)F * c->S * c->n_bc;
  if (need <= c->body_pair_cap) return;
  void* pp = c->body_pair;
  c->release(pp);
  c->body_pair = nullptr;
  c->body_pair_cap = 0;
  c->body_pair = (int*)c->alloc(need * sizeof(int));
  c->body_pair_cap = need;
}

// per-frame checkpoints of (x, v) for F frames
void ensure_checkpoints(xpbd_ctx c, int F) {
  if (c->ck_frames >= F) return;
  const size_t vb = (size_t)c->V * 4 * c->tsz;
  c->release(c->ckX);
  c->release(c->ckV);
  c->ck_frames = 0;
  c->ckX = c->alloc((size_t)F * vb);
  c->ckV = c->alloc((size_t)F * vb);
  c->ck_frames = F;
}

template <class T> struct Ops {
  using V4 = Vec4<T>;

  static void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(XPBD_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  }

  static Dev<T> dev(xpbd_ctx c, const double* s) {
    Dev<T> D{};
    D.X = (V4*)c->X; D.Vv = (V4*)c->Vv; D.Xp = (V4*)c->Xp; D.XB = (V4*)c->XB; D.VB = (V4*)c->VB; D.V = c->V;
    D.d_idx = c->dist_idx; D.d_rest = (const T*)c->dist_rest; D.d_at = (const T*)c->dist_at;
    D.d_lam = (T*)c->dist_lam; D.d_lamb = (T*)c->dist_lamb; D.d_ab = (T*)c->dist_ab; D.d_acc = c->dist_acc;
    D.b_idx = c->bend_idx; D.b_th0 = (const T*)c->bend_theta0; D.b_at = (const T*)c->bend_at;
    D.b_lam = (T*)c->bend_lam; D.b_lamb = (T*)c->bend_lamb; D.b_ab = (T*)c->bend_ab; D.b_acc = c->bend_acc;
    D.tr = TetRec<T>{c->tet_idx, (const T*)c->tet_B, (const T*)c->tet_atD, (const T*)c->tet_atH,
                     (const T*)c->tet_gamma, c->n_tet};
    D.t_lamD = (T*)c->tet_lamD; D.t_lamH = (T*)c->tet_lamH; D.t_lambD = (T*)c->tet_lambD;
    D.t_lambH = (T*)c->tet_lambH; D.t_eb = (T*)c->tet_eb; D.t_acc = c->tet_acc;
    D.c_vid = c->contact_vid; D.c_lam = (T*)c->contact_lam; D.c_lamb = (T*)c->contact_lamb;
    D.c_sacc = (V4*)c->contact_sacc;
    D.c_order = c->contact_order;
    D.mr = TriRec<T>{c->tri_idx, (const T*)c->tri_B, (const T*)c->tri_at, c->n_tri};
    D.m_lam = (T*)c->tri_lam; D.m_lamb = (T*)c->tri_lamb; D.m_ab = (T*)c->tri_ab; D.m_acc = c->tri_acc;
    D.bc_vid = c->bc_vid; D.bc_lam = (T*)c->bc_lam; D.bc_lamb = (T*)c->bc_lamb; D.bpair = nullptr;
    D.bx = (const T*)c->cur_body_x; D.btri = c->body_tris; D.bgrad = nullptr;
    D.bc_tau = (T)c->b_tau; D.bc_at = (T)(c->b_alpha / (c->h * c->h));
    D.sph = Sphere<T>{(T)s[0], (T)s[1], (T)s[2], (T)s[3], (T)c->tau, (T)(c->alpha_c / (c->h * c->h))};
    D.h = (T)c->h; D.inv_h = (T)(1.0 / c->h);
    D.gx = (T)c->g[0]; D.gy = (T)c->g[1]; D.gz = (T)c->g[2];
    return D;
  }

  // ------------------------------------------------------------ plain launches (one per set)
  static void project(xpbd_ctx c, const Dev<T>* D, const SetInfo& si, bool first, V4* tape, hipStream_t st) {
    if (si.count == 0) return;
    const int bs = c->block;
    unsigned nb = nblocks(si.count, bs);
    xpbd_ctx_s::Ev ev;
    bool on;
    prof_begin(c, st, prof_family(si.type, false), si.type == XPBD_TET ? 2 * (int64_t)si.count : si.count, &ev,
               &on);
#define XPBD_LAUNCH(KERN, TP)                                                                     \
  do {                                                                                            \
    if (first) {                                                                                  \
      if (tape) KERN<T, true, true><<<nb, bs, 0, st>>>(D, si.begin, si.count, (TP*)tape);         \
      else KERN<T, true, false><<<nb, bs, 0, st>>>(D, si.begin, si.count, (TP*)tape);             \
    } else {                                                                                      \
      if (tape) KERN<T, false, true><<<nb, bs, 0, st>>>(D, si.begin, si.count, (TP*)tape);        \
      else KERN<T, false, false><<<nb, bs, 0, st>>>(D, si.begin, si.count, (TP*)tape);            \
    }                                                                                             \
  } while (0)
    switch (si.type) {
      case XPBD_DIST: XPBD_LAUNCH(k_dist, V4); break;
      case XPBD_BEND: XPBD_LAUNCH(k_bend, V4); break;
      case XPBD_TET: XPBD_LAUNCH(k_tet, V4); break;
      case XPBD_TRI: XPBD_LAUNCH(k_tri, V4); break;
      case XPBD_BODY: XPBD_LAUNCH(k_body, V4); break;
      default: XPBD_LAUNCH(k_contact, V4); break;
    }
    check_launch();
    prof_end(c, st, ev, on);
  }

  static void reverse(xpbd_ctx c, const Dev<T>* D, const SetInfo& si, bool first, bool last, const V4* tape,
                      hipStream_t st) {
    if (si.count == 0) return;
    const int bs = c->block;
    unsigned nb = nblocks(si.count, bs);
    xpbd_ctx_s::Ev ev;
    bool on;
    prof_begin(c, st, prof_family(si.type, true), si.type == XPBD_TET ? 2 * (int64_t)si.count : si.count, &ev,
               &on);
    const bool tape_ = last;   // second template flag of the reverse kernels is LAST
    (void)tape_;
#define XPBD_RLAUNCH(KERN)                                                                        \
  do {                                                                                            \
    if (first) {                                                                                  \
      if (last) KERN<T, true, true><<<nb, bs, 0, st>>>(D, si.begin, si.count, tape);              \
      else KERN<T, true, false><<<nb, bs, 0, st>>>(D, si.begin, si.count, tape);                  \
    } else {                                                                                      \
      if (last) KERN<T, false, true><<<nb, bs, 0, st>>>(D, si.begin, si.count, tape);             \
      else KERN<T, false, false><<<nb, bs, 0, st>>>(D, si.begin, si.count, tape);                 \
    }                                                                                             \
  } while (0)
    switch (si.type) {
      case XPBD_DIST: XPBD_RLAUNCH(k_dist_rev); break;
      case XPBD_BEND: XPBD_RLAUNCH(k_bend_rev); break;
      case XPBD_TET: XPBD_RLAUNCH(k_tet_rev); break;
      case XPBD_TRI: XPBD_RLAUNCH(k_tri_rev); break;
      case XPBD_BODY: XPBD_RLAUNCH(k_body_rev); break;
      default: XPBD_RLAUNCH(k_contact_rev); break;
    }
#undef XPBD_LAUNCH
#undef XPBD_RLAUNCH
    check_launch();
    prof_end(c, st, ev, on);
  }

  // record pointer of set si, iteration it, substep slot (within the record buffer)
  static V4* tape_at(xpbd_ctx c, int slot, int it, const SetInfo& si) {
    char* base = (char*)c->tape + ((size_t)slot * c->K + it) * c->iter_tape_bytes + si.tape_off;
    return (V4*)base;
  }

  static GroupDev group_dev(const xpbd_ctx_s::Group& g) {
    GroupDev G;
    G.pv_start = g.pv_start; G.pv = g.pv; G.cnt = g.cnt; G.set_type = g.set_type;
    G.img = g.img; G.fmul = g.fmul; G.rmul = g.rmul; G.tpos = g.tpos; G.rec_first = g.rec_first;
    G.nset = g.b - g.a;
    G.P = g.P;
    G.tape_off = g.tape_off;
    G.snap_x_off = g.snap_x_off;
    G.snap_l_off = g.snap_l_off;
    G.fmul_lo = g.fmul_lo;
    return G;
  }

  static void group_fwd(xpbd_ctx c, const Dev<T>& D, const xpbd_ctx_s::Group& g, bool first, char* tape_iter,
                        hipStream_t st) {
    GroupDev G = group_dev(g);
    xpbd_ctx_s::Ev ev;
    bool on;
    prof_begin(c, st, 10, g.items, &ev, &on);
    dim3 grid(g.P);
    const bool rl = !c->group_stream;
    const int bs = c->group_block;
    const size_t sm = rl ? g.smem_fwd : g.smem_tile;
#define XPBD_GF(F1, F2)                                                                             \
  do {                                                                                              \
    if (rl && g.heavy) k_group_fwd<T, F1, F2, true, true><<<grid, bs, sm, st>>>(D, G, c->gimg, c->gfmul, tape_iter);   \
    else if (rl) k_group_fwd<T, F1, F2, true, false><<<grid, bs, sm, st>>>(D, G, c->gimg, c->gfmul, tape_iter);  \
    else if (g.heavy) k_group_fwd<T, F1, F2, false, true><<<grid, bs, sm, st>>>(D, G, c->gimg, c->gfmul, tape_iter); \
    else k_group_fwd<T, F1, F2, false, false><<<grid, bs, sm, st>>>(D, G, c->gimg, c->gfmul, tape_iter);         \
  } while (0)
    // REC: 0 no record, 1 every projection's inputs, 2 a snapshot of the launch's inputs
    const int rec = !tape_iter ? 0 : c->record_kind == 1 ? 2 : 1;
    if (first) {
      if (rec == 2) XPBD_GF(true, 2);
      else if (rec == 1) XPBD_GF(true, 1);
      else XPBD_GF(true, 0);
    } else {
      if (rec == 2) XPBD_GF(false, 2);
      else if (rec == 1) XPBD_GF(false, 1);
      else XPBD_GF(false, 0);
    }
#undef XPBD_GF
    check_launch();
    prof_end(c, st, ev, on);
  }

  static void group_rev(xpbd_ctx c, const Dev<T>& D, const xpbd_ctx_s::Group& g, bool first, bool last,
                        const char* tape_iter, hipStream_t st) {
    GroupDev G = group_dev(g);
    xpbd_ctx_s::Ev ev;
    bool on;
    prof_begin(c, st, 11, g.items, &ev, &on);
    dim3 grid(g.P);
    const bool rl = !c->group_stream;
    const int bs = c->group_block;
    // replay the launch from its snapshot: 0 no, 1 record to the scratch, 2 record in LDS
    const int rp = c->record_kind != 1 ? 0 : (rl || g.replay_lds) ? 2 : 1;
    const size_t sm = rl ? g.smem_rev + (rp ? g.smem_tile : 0)
                         : g.smem_tile + (rp ? g.smem_tile : 0) + (rp == 2 ? g.max_tbytes : 0);
    char* scr = c->scratch;
    // no distance / bending compliance gradient asked for: the variant
    // without those adjoints (distance, bending and contact groups, records
    // of projection inputs)
    const bool no_ab = !c->want_ab && !g.heavy && rp == 0;
#define XPBD_GR(F1, F2, RP)                                                                         \
  do {                                                                                              \
    if (rl && g.heavy) k_group_rev<T, F1, F2, true, true, RP><<<grid, bs, sm, st>>>(D, G, c->gimg, c->grmul, tape_iter, scr);   \
    else if (rl) k_group_rev<T, F1, F2, true, false, RP><<<grid, bs, sm, st>>>(D, G, c->gimg, c->grmul, tape_iter, scr);  \
    else if (g.heavy) k_group_rev<T, F1, F2, false, true, RP><<<grid, bs, sm, st>>>(D, G, c->gimg, c->grmul, tape_iter, scr); \
    else k_group_rev<T, F1, F2, false, false, RP><<<grid, bs, sm, st>>>(D, G, c->gimg, c->grmul, tape_iter, scr);         \
  } while (0)
#define XPBD_GR3(F1, F2)                                  \
  do {                                                    \
    if (no_ab && rl) k_group_rev<T, F1, F2, true, false, 0, false><<<grid, bs, sm, st>>>(D, G, c->gimg, c->grmul, tape_iter, scr); \
    else if (no_ab) k_group_rev<T, F1, F2, false, false, 0, false><<<grid, bs, sm, st>>>(D, G, c->gimg, c->grmul, tape_iter, scr); \
    else if (rp == 2) XPBD_GR(F1, F2, 2);                 \
    else if (rp == 1) XPBD_GR(F1, F2, 1);                 \
    else XPBD_GR(F1, F2, 0);                              \
  } while (0)
    if (first) {
      if (last) XPBD_GR3(true, true);
      else XPBD_GR3(true, false);
    } else {
      if (last) XPBD_GR3(false, true);
      else XPBD_GR3(false, false);
    }
#undef XPBD_GR3
#undef XPBD_GR
    check_launch();
    prof_end(c, st, ev, on);
  }

  static void group_fill(xpbd_ctx c, hipStream_t st) {
    if (!c->gimg) return;
    if (c->n_dist && c->gpos[0])
      k_group_fill<T><<<nblocks(c->n_dist), kBlock, 0, st>>>(0, c->n_dist, c->gpos[0], c->gimg,
                                                             (const T*)c->dist_at, nullptr, nullptr);
    if (c->n_bend && c->gpos[1])
      k_group_fill<T><<<nblocks(c->n_bend), kBlock, 0, st>>>(1, c->n_bend, c->gpos[1], c->gimg,
                                                             (const T*)c->bend_at, nullptr, nullptr);
    if (c->n_tet && c->gpos[2])
      k_group_fill<T><<<nblocks(c->n_tet), kBlock, 0, st>>>(2, c->n_tet, c->gpos[2], c->gimg,
                                                            (const T*)c->tet_atD, (const T*)c->tet_atH,
                                                            (const T*)c->tet_gamma);
    if (c->n_tri && c->gpos[3])
      k_group_fill<T><<<nblocks(c->n_tri), kBlock, 0, st>>>(4, c->n_tri, c->gpos[3], c->gimg,
                                                            (const T*)c->tri_at, nullptr, nullptr);
    check_launch();
  }

  static void allow_lds(size_t bytes) {
    if (bytes <= 65536) return;
    allow_lds_heavy<true>(bytes);
    allow_lds_heavy<false>(bytes);
  }
  template <bool HEAVY> static void allow_lds_heavy(size_t bytes) {
    const void* ks[] = {
#define XPBD_FWD_K(F1, RL) (const void*)k_group_fwd<T, F1, 0, RL, HEAVY>, (const void*)k_group_fwd<T, F1, 1, RL, HEAVY>, \
                           (const void*)k_group_fwd<T, F1, 2, RL, HEAVY>
#define XPBD_REV_K(F1, F2, RL) (const void*)k_group_rev<T, F1, F2, RL, HEAVY, 0>, \
                               (const void*)k_group_rev<T, F1, F2, RL, HEAVY, 1>, \
                               (const void*)k_group_rev<T, F1, F2, RL, HEAVY, 2>
        XPBD_FWD_K(true, true), XPBD_FWD_K(false, true), XPBD_FWD_K(true, false), XPBD_FWD_K(false, false),
        XPBD_REV_K(true, true, true), XPBD_REV_K(true, false, true), XPBD_REV_K(false, true, true),
        XPBD_REV_K(false, false, true), XPBD_REV_K(true, true, false), XPBD_REV_K(true, false, false),
        XPBD_REV_K(false, true, false), XPBD_REV_K(false, false, false),
        (const void*)k_group_rev<T, true, true, true, false, 0, false>,
        (const void*)k_group_rev<T, true, false, true, false, 0, false>,
        (const void*)k_group_rev<T, false, true, true, false, 0, false>,
        (const void*)k_group_rev<T, false, false, true, false, 0, false>};
#undef XPBD_FWD_K
#undef XPBD_REV_K
    for (const void* k : ks) HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }

  // device copy `which` of the per-set kernels' parameter block
  static Dev<T>* dev_block(xpbd_ctx c, int which) {
    static_assert(sizeof(Dev<T>) <= kDevBlk, "parameter block larger than its device slot");
    return (Dev<T>*)((char*)c->dev_blk + (size_t)which * kDevBlk);
  }

  // body pairing of global substep gsub (frame * S + substep)
  static int* pairs_of(xpbd_ctx c, int gsub) {
    if (!c->n_bc) return nullptr;
    if (gsub < 0 || (size_t)(gsub + 1) * c->n_bc > c->body_pair_cap) fail(XPBD_ERR_STATE, "body pairing slot");
    return c->body_pair + (size_t)gsub * c->n_bc;
  }

  // one substep of Eq. xpbdUpdateRule; record slot < 0 means no record;
  // gsub = frame * S + substep (the body pairing's slot)
  static void substep(xpbd_ctx c, const Dev<T>& D0, const T* f, int slot, hipStream_t st, int gsub = -1) {
    Range range_(slot >= 0 ? "xpbd substep (recording)" : "xpbd substep");
    Dev<T> D = D0;
    k_predict<T><<<nblocks(c->V), kBlock, 0, st>>>(D, f);
    check_launch();
    if (c->n_bc) {
      D.bpair = pairs_of(c, gsub);
      k_body_detect<T><<<nblocks(c->n_bc), kBlock, 0, st>>>((const V4*)c->X, c->bc_vid, c->n_bc, D.bx, c->body_tris,
                                                            c->grid, c->b_radius * c->b_radius, (int*)D.bpair);
      check_launch();
    }
    Dev<T>* blk = dev_block(c, 0);
    k_store_dev<T><<<1, 64, 0, st>>>(D, blk);
    check_launch();
    const int ns = (int)c->sets.size();
    for (int it = 0; it < c->K; ++it) {
      Range sweep_("xpbd sweep");
      for (int k = 0; k < ns; ++k) {
        int g = c->group_at_start.empty() ? -1 : c->group_at_start[k];
        if (g >= 0 && c->groups[g].lds) {
          char* ti = slot >= 0 ? (char*)c->tape + ((size_t)slot * c->K + it) * c->iter_tape_bytes : nullptr;
          group_fwd(c, D, c->groups[g], it == 0, ti, st);
          k = c->groups[g].b - 1;
          continue;
        }
        const SetInfo& si = c->sets[k];
        project(c, blk, si, it == 0, slot >= 0 ? tape_at(c, slot, it, si) : nullptr, st);
      }
    }
    k_velocity<T><<<nblocks(c->V), kBlock, 0, st>>>(D);
    check_launch();
  }

  static void reverse_substep(xpbd_ctx c, const Dev<T>& D0, T* fbar, double* dsph, int slot, hipStream_t st,
                              int gsub = -1) {
    Range range_("xpbd reverse substep");
    Dev<T> D = D0;
    if (c->n_bc) D.bpair = pairs_of(c, gsub);
    Dev<T>* blk = dev_block(c, 1);
    k_store_dev<T><<<1, 64, 0, st>>>(D, blk);
    check_launch();
    k_rev_velocity<T><<<nblocks(c->V), kBlock, 0, st>>>(D);
    check_launch();
    for (int it = c->K - 1; it >= 0; --it) {
      Range sweep_("xpbd reverse sweep");
      for (int k = (int)c->sets.size() - 1; k >= 0; --k) {
        int g = c->group_at_end.empty() ? -1 : c->group_at_end[k];
        if (g >= 0 && c->groups[g].lds) {
          const char* ti = (const char*)c->tape + ((size_t)slot * c->K + it) * c->iter_tape_bytes;
          group_rev(c, D, c->groups[g], it == c->K - 1, it == 0, ti, st);
          k = c->groups[g].a;
          continue;
        }
        const SetInfo& si = c->sets[k];
        reverse(c, blk, si, it == c->K - 1, it == 0, tape_at(c, slot, it, si), st);
      }
    }
    if (c->K > 0 && dsph)
      for (const SetInfo& si : c->sets)
        if (si.type == XPBD_CONTACT && si.count > 0) {
          k_sphere_reduce<T><<<1, kBlock, 0, st>>>((const V4*)c->contact_sacc, c->contact_order, si.begin, si.count,
                                                   dsph);
          check_launch();
        }
    k_rev_predict<T><<<nblocks(c->V), kBlock, 0, st>>>(D, fbar);
    check_launch();
  }

  // ------------------------------------------------------------ persistent program launches
  // Forward program of one frame: S x (predict, K x sets, velocity), record
  // offsets relative to the frame's record base; reverse program mirrors it.
  static void build_programs(xpbd_ctx c) {
    std::vector<Phase> fw, rv;
    const int S = c->S, K = c->K;
    for (int s = 0; s < S; ++s) {
      fw.push_back({OP_PREDICT, 0, 0, c->V, -1});
      for (int it = 0; it < K; ++it)
        for (const SetInfo& si : c->sets) {
          if (!si.count) continue;
          long long off = (long long)(((size_t)s * K + it) * c->iter_tape_bytes + si.tape_off);
          fw.push_back({OP_SET + si.type, (it == 0 ? PF_FIRST : 0) | PF_SECOND, si.begin, si.count, off});
        }
      fw.push_back({OP_VELOCITY, 0, 0, c->V, -1});
    }
    for (int s = S - 1; s >= 0; --s) {
      rv.push_back({OP_REV_VELOCITY, 0, 0, c->V, -1});
      for (int it = K - 1; it >= 0; --it)
        for (int k = (int)c->sets.size() - 1; k >= 0; --k) {
          const SetInfo& si = c->sets[k];
          if (!si.count) continue;
          long long off = (long long)(((size_t)s * K + it) * c->iter_tape_bytes + si.tape_off);
          rv.push_back({OP_SET_REV + si.type, (it == K - 1 ? PF_FIRST : 0) | (it == 0 ? PF_SECOND : 0), si.begin,
                        si.count, off});
        }
      if (K > 0)
        for (const SetInfo& si : c->sets)
          if (si.type == XPBD_CONTACT && si.count) rv.push_back({OP_SPHERE, 0, si.begin, si.count, -1});
      rv.push_back({OP_REV_PREDICT, 0, 0, c->V, -1});
    }
    c->n_fw_prog = (int)fw.size();
    c->n_rv_prog = (int)rv.size();
    c->fw_prog = (Phase*)c->alloc(fw.size() * sizeof(Phase));
    c->rv_prog = (Phase*)c->alloc(rv.size() * sizeof(Phase));
    c->upload(c->fw_prog, fw);
    c->upload(c->rv_prog, rv);
  }

  static int program_grid(xpbd_ctx c) {
    if (c->prog_grid) return c->prog_grid;
    int dev = 0, ncu = 0, per_cu = 0, coop = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) fail(XPBD_ERR_HIP, "device does not support cooperative launch");
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_program<T>, kBlock, 0));
    int cap = ncu * std::max(per_cu, 1);
    int want = c->prog_blocks_opt;
    if (want <= 0) {
      int mx = c->V;
      for (const SetInfo& si : c->sets) mx = std::max(mx, si.count);
      want = (int)nblocks(mx);
    }
    c->prog_grid = std::max(1, std::min(std::min(want, cap), 4096));
    return c->prog_grid;
  }

  static void run_program(xpbd_ctx c, const Dev<T>& D, bool reverse_prog, char* tape_base, const T* f, T* fbar,
                          double* dsph, bool record, hipStream_t st) {
    if (!c->fw_prog) build_programs(c);
    int G = program_grid(c);
    RunArgs<T> R{};
    R.tape = tape_base;
    R.f = f;
    R.fbar = fbar;
    R.sph_out = dsph;
    R.record = record ? 1 : 0;
    R.bar = c->bar;
    R.abort = c->abort_flag;
    R.spin_limit = 1u << 22;
    const Phase* prog = reverse_prog ? c->rv_prog : c->fw_prog;
    int n = reverse_prog ? c->n_rv_prog : c->n_fw_prog;
    if (n == 0) return;
    HIPCHK(hipMemsetAsync(c->bar, 0, ((size_t)G * kFlagStride + 1) * sizeof(unsigned), st));
    Dev<T> Dl = D;
    void* args[] = {(void*)&Dl, (void*)&prog, (void*)&n, (void*)&R};
    xpbd_ctx_s::Ev ev;
    bool on;
    prof_begin(c, st, reverse_prog ? 9 : 8, (int64_t)c->S * c->K * c->proj_per_iter, &ev, &on);
    HIPCHK(hipLaunchCooperativeKernel((const void*)k_program<T>, dim3(G), dim3(kBlock), args, 0, st));
    prof_end(c, st, ev, on);
  }

  // ------------------------------------------------------------ frame loops
  // The pairing grid of the body in its current position (host, FP64):
  // cells of edge >= the search radius over the body's box grown by it.
  static void build_body_grid(xpbd_ctx c, const T* bx_dev, hipStream_t st) {
    const int nv = c->body_nv, nt = c->body_nt;
    std::vector<T> bt((size_t)3 * nv);
    HIPCHK(hipMemcpyAsync(bt.data(), bx_dev, bt.size() * sizeof(T), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<double> b(bt.begin(), bt.end());
    for (double v : b)
      if (!std::isfinite(v)) fail(XPBD_ERR_NONFINITE, "body vertex position not finite");
    const double r = c->b_radius;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = 1e300; hi[a] = -1e300; }
    for (int k = 0; k < nv; ++k)
      for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], b[3 * k + a]); hi[a] = std::max(hi[a], b[3 * k + a]); }
    double ext = 0;
    for (int a = 0; a < 3; ++a) { lo[a] -= r; hi[a] += r; ext = std::max(ext, hi[a] - lo[a]); }
    const double cell = std::max(r, ext / 64.0);
    int dims[3];
    for (int a = 0; a < 3; ++a) dims[a] = std::max(1, (int)std::ceil((hi[a] - lo[a]) / cell));
    const size_t ncell = (size_t)dims[0] * dims[1] * dims[2];
    auto cell_range = [&](int t, int a, int& i0, int& i1) {
      double mn = 1e300, mx = -1e300;
      for (int j = 0; j < 3; ++j) {
        double v = b[3 * (size_t)c->body_tris_h[3 * (size_t)t + j] + a];
        mn = std::min(mn, v);
        mx = std::max(mx, v);
      }
      i0 = std::max(0, (int)std::floor((mn - r - lo[a]) / cell));
      i1 = std::min(dims[a] - 1, (int)std::floor((mx + r - lo[a]) / cell));
    };
    std::vector<int> off(ncell + 1, 0);
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int> fillp;
      std::vector<int> lists;
      if (pass == 1) {
        for (size_t q = 0; q < ncell; ++q) off[q + 1] += off[q];
        fillp.assign(off.begin(), off.end() - 1);
        lists.resize(off[ncell]);
      }
      for (int t = 0; t < nt; ++t) {
        int r0[3], r1[3];
        for (int a = 0; a < 3; ++a) cell_range(t, a, r0[a], r1[a]);
        for (int i = r0[0]; i <= r1[0]; ++i)
          for (int j = r0[1]; j <= r1[1]; ++j)
            for (int k = r0[2]; k <= r1[2]; ++k) {
              size_t q = ((size_t)i * dims[1] + j) * dims[2] + k;
              if (pass == 0) ++off[q + 1];
              else lists[fillp[q]++] = t;
            }
      }
      if (pass == 1) {
        if (off.size() > c->grid_off_cap) {
          void* pp = c->grid_off;
          c->release(pp);
          c->grid_off = (int*)c->alloc(off.size() * sizeof(int));
          c->grid_off_cap = off.size();
        }
        if (std::max<size_t>(lists.size(), 1) > c->grid_tris_cap) {
          void* pp = c->grid_tris;
          c->release(pp);
          c->grid_tris = (int*)c->alloc(std::max<size_t>(lists.size(), 1) * sizeof(int));
          c->grid_tris_cap = std::max<size_t>(lists.size(), 1);
        }
        c->upload(c->grid_off, off);
        c->upload(c->grid_tris, lists);
      }
    }
    for (int a = 0; a < 3; ++a) { c->grid.lo[a] = lo[a]; c->grid.dims[a] = dims[a]; }
    c->grid.inv_cell = 1.0 / cell;
    c->grid.off = c->grid_off;
    c->grid.tris = c->grid_tris;
  }

  template <class U> static void fill(U* p, U v, size_t n, hipStream_t st) {
    if (!n || !p) return;
    k_fill<U><<<nblocks(n), kBlock, 0, st>>>(p, v, n);
    check_launch();
  }

  static void gather_params(xpbd_ctx c, const xpbd_params* p, hipStream_t st) {
    HIPCHK(hipMemsetAsync(c->flag, 0, sizeof(int), st));
    double ih2 = 1.0 / (c->h * c->h);
    if (c->n_dist)
      k_gather_alpha<T><<<nblocks(c->n_dist), kBlock, 0, st>>>((const T*)p->dist_compliance, c->dist_perm,
                                                               (T*)c->dist_at, (T)ih2, c->n_dist, c->flag);
    if (c->n_bend)
      k_gather_alpha<T><<<nblocks(c->n_bend), kBlock, 0, st>>>((const T*)p->bend_compliance, c->bend_perm,
                                                               (T*)c->bend_at, (T)ih2, c->n_bend, c->flag);
    if (c->n_tet) {
      if (p->tet_mu)
        k_gather_tet_lame<T><<<nblocks(c->n_tet), kBlock, 0, st>>>((const T*)p->tet_mu, (const T*)p->tet_lambda,
                                                                   c->tet_pidx, c->tet_vol, (T*)c->tet_atD,
                                                                   (T*)c->tet_atH, (T*)c->tet_gamma, ih2,
                                                                   c->gamma_one, c->n_tet, c->flag);
      else
        k_gather_tet<T><<<nblocks(c->n_tet), kBlock, 0, st>>>((const T*)p->tet_E, c->tet_pidx, c->tet_nu,
                                                            c->tet_vol, (T*)c->tet_atD, (T*)c->tet_atH,
                                                            (T*)c->tet_gamma, ih2, c->gamma_one, c->n_tet, c->flag);
    }
    if (c->n_tri)
      k_gather_tri<T><<<nblocks(c->n_tri), kBlock, 0, st>>>((const T*)p->tri_coef, c->tri_perm, c->tri_area,
                                                            (T*)c->tri_at, ih2, c->n_tri, c->flag);
    c->cur_body_x = p->body_x;
    if (c->n_bc) build_body_grid(c, (const T*)p->body_x, st);
    check_launch();
    group_fill(c, st);
    int flags[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&flags[0], c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&flags[1], c->abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flags[1]) {
      HIPCHK(hipMemset(c->abort_flag, 0, sizeof(int)));
      fail(XPBD_ERR_HIP, "an earlier persistent sweep gave up waiting at a grid barrier; its results are invalid");
    }
    if (flags[0]) fail(XPBD_ERR_NONFINITE, "a compliance or Young's modulus is negative, zero (E) or not finite");
    for (int a = 0; a < 4; ++a)
      if (!std::isfinite(p->sphere[a])) fail(XPBD_ERR_NONFINITE, "sphere parameter %d is not finite", a);
  }

  // frames f >= rec_from keep their record in slot (f - rec_from) (rec_from = F: none)
  static void forward(xpbd_ctx c, const void* x0, const void* v0, const xpbd_params* p, int F, void* xf,
                      void* x_final, void* v_final, int rec_from, hipStream_t st) {
    const int V = c->V;
    const size_t vb = (size_t)V * sizeof(V4);
    ensure_checkpoints(c, F);
    ensure_body_pairs(c, F);
    gather_params(c, p, st);
    Dev<T> D = dev(c, p->sphere);
    k_pack<T><<<nblocks(V), kBlock, 0, st>>>((const T*)x0, (const T*)v0, (const T*)c->w, (V4*)c->X, (V4*)c->Vv, V);
    check_launch();
    const size_t frame_tape = (size_t)c->S * c->K * c->iter_tape_bytes;
    for (int f = 0; f < F; ++f) {
      Range frame_("xpbd frame");
      HIPCHK(hipMemcpyAsync((char*)c->ckX + f * vb, c->X, vb, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync((char*)c->ckV + f * vb, c->Vv, vb, hipMemcpyDeviceToDevice, st));
      const T* ff = p->f_ext ? (const T*)p->f_ext + (size_t)f * 3 * V : nullptr;
      const bool record = f >= rec_from;
      const int fr = f - rec_from;
      if (c->persistent) {
        run_program(c, D, false, record ? (char*)c->tape + (size_t)fr * frame_tape : nullptr, ff, nullptr, nullptr,
                    record, st);
      } else {
        for (int s = 0; s < c->S; ++s) substep(c, D, ff, record ? fr * c->S + s : -1, st, f * c->S + s);
      }
      if (xf) {
        k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->X, (T*)xf + (size_t)f * 3 * V, V);
        check_launch();
      }
    }
    if (x_final) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->X, (T*)x_final, V);
    if (v_final) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->Vv, (T*)v_final, V);
    check_launch();
  }

  static void restore(xpbd_ctx c, int f, hipStream_t st) {
    const size_t vb = (size_t)c->V * sizeof(V4);
    HIPCHK(hipMemcpyAsync(c->X, (char*)c->ckX + f * vb, vb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c->Vv, (char*)c->ckV + f * vb, vb, hipMemcpyDeviceToDevice, st));
  }

  // frames f >= rec_from use the record the forward kept (slot f - rec_from);
  // the others are recomputed per frame (mode 1) or per substep (mode 2)
  static void adjoint(xpbd_ctx c, const xpbd_params* p, const void* dLdx, const uint8_t* mask, const void* dLdv,
                      const xpbd_grads* out, int mode, int rec_from, hipStream_t st) {
    const int V = c->V, F = c->fwd_frames, S = c->S;
    // parameters used by the recomputation (same as the forward's)
    gather_params(c, p, st);
    begin_adjoint(c, F, dLdv, out, st);
    Dev<T> D = dev(c, p->sphere);
    D.bgrad = out->body_x;
    const size_t frame_tape = (size_t)S * c->K * c->iter_tape_bytes;
    const int nslot = frame_tape ? (int)std::min<size_t>(c->tape_cap / frame_tape, (size_t)F) : 0;
    c->adj_streams_used = 1;
    if (!c->persistent && !c->serial_adjoint && mode == 1 && rec_from > 0 && nslot >= 2) {
      c->adj_streams_used = 2;
      adjoint_overlapped(c, p, D, dLdx, mask, out, rec_from, nslot, st);
      finish_adjoint(c, p, out, st);
      return;
    }
    for (int f = F - 1; f >= 0; --f) {
      Range frame_("xpbd adjoint frame");
      if (dLdx && (!mask || mask[f])) {
        k_adj_inject<T><<<nblocks(V), kBlock, 0, st>>>((V4*)c->XB, (const T*)dLdx + (size_t)f * 3 * V, V);
        check_launch();
      }
      const T* ff = p->f_ext ? (const T*)p->f_ext + (size_t)f * 3 * V : nullptr;
      T* fb = out->f_ext ? (T*)out->f_ext + (size_t)f * 3 * V : nullptr;
      const bool kept = f >= rec_from;
      if (kept || mode == 1) {
        char* base = kept ? (char*)c->tape + (size_t)(f - rec_from) * frame_tape : (char*)c->tape;
        if (!kept) {
          restore(c, f, st);
          if (c->persistent) run_program(c, D, false, base, ff, nullptr, nullptr, true, st);
          else for (int s = 0; s < S; ++s) substep(c, D, ff, s, st, f * S + s);
        }
        if (c->persistent) {
          run_program(c, D, true, base, nullptr, fb, out->sphere, false, st);
        } else {
          int slot0 = kept ? (f - rec_from) * S : 0;
          for (int s = S - 1; s >= 0; --s) reverse_substep(c, D, fb, out->sphere, slot0 + s, st, f * S + s);
        }
      } else {
        for (int s = S - 1; s >= 0; --s) {
          restore(c, f, st);
          for (int q = 0; q < s; ++q) substep(c, D, ff, -1, st, f * S + q);
          substep(c, D, ff, 0, st, f * S + s);
          reverse_substep(c, D, fb, out->sphere, 0, st, f * S + s);
        }
      }
    }
    finish_adjoint(c, p, out, st);
  }

  // Adjoint with the recomputation of earlier frames beside the reverse.
  // The record holds nslot frames: the kept frames f >= rec_from in slot
  // f - rec_from, the others free.  A recomputed frame g takes the slot of
  // frame g + nslot once that frame has been reversed (or a free slot), so
  // its recomputation on one library stream runs while the frames between
  // are reversed on another.  The recomputation touches only the forward
  // state (positions, velocities, multipliers, forward group state) and its
  // slot; the reverse only the adjoint state, the gradient outputs and the
  // slots of frames already recorded.  Events order each reverse after its
  // frame's recomputation and each slot's reuse after the reverse that read
  // it; the call's stream waits for both streams at the start and for the
  // reverse stream at the end.  Every kernel sees the same inputs as in the
  // serial order, so the results are bitwise those of one stream.
  static void adjoint_overlapped(xpbd_ctx c, const xpbd_params* p, const Dev<T>& D, const void* dLdx,
                                 const uint8_t* mask, const xpbd_grads* out, int rec_from, int nslot,
                                 hipStream_t st) {
    const int V = c->V, F = c->fwd_frames, S = c->S;
    if (!c->adj_rec) HIPCHK(hipStreamCreateWithFlags(&c->adj_rec, hipStreamNonBlocking));
    if (!c->adj_rev) HIPCHK(hipStreamCreateWithFlags(&c->adj_rev, hipStreamNonBlocking));
    hipStream_t sr = c->adj_rec, sv = c->adj_rev;
    // events: [0, F) frame recomputed, [F, 2F) frame reversed, start, end
    while (c->adj_events.size() < (size_t)2 * F + 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->adj_events.push_back(e);
    }
    hipEvent_t* ev_rec = c->adj_events.data();
    hipEvent_t* ev_rev = ev_rec + F;
    hipEvent_t ev_start = ev_rec[2 * F], ev_end = ev_rec[2 * F + 1];
    const int kept_n = F - rec_from;
    std::vector<int> slot(F, -1);
    for (int f = rec_from; f < F; ++f) slot[f] = f - rec_from;
    for (int g = rec_from - 1; g >= 0; --g)
      slot[g] = g + nslot <= F - 1 ? slot[g + nslot] : kept_n + (rec_from - 1 - g);
    HIPCHK(hipEventRecord(ev_start, st));
    HIPCHK(hipStreamWaitEvent(sr, ev_start, 0));
    HIPCHK(hipStreamWaitEvent(sv, ev_start, 0));
    int next = rec_from - 1;   // next frame to recompute, descending
    for (int f = F - 1; f >= 0; --f) {
      // enqueue every recomputation whose slot is free once the reverses
      // enqueued so far have run
      while (next >= 0 && next + nslot > f) {
        const int g = next--;
        Range rec_("xpbd recompute frame");
        if (g + nslot <= F - 1) HIPCHK(hipStreamWaitEvent(sr, ev_rev[g + nslot], 0));
        const T* fg = p->f_ext ? (const T*)p->f_ext + (size_t)g * 3 * V : nullptr;
        restore(c, g, sr);
        for (int s = 0; s < S; ++s) substep(c, D, fg, slot[g] * S + s, sr, g * S + s);
        HIPCHK(hipEventRecord(ev_rec[g], sr));
      }
      Range frame_("xpbd adjoint frame");
      if (f < rec_from) HIPCHK(hipStreamWaitEvent(sv, ev_rec[f], 0));
      if (dLdx && (!mask || mask[f])) {
        k_adj_inject<T><<<nblocks(V), kBlock, 0, sv>>>((V4*)c->XB, (const T*)dLdx + (size_t)f * 3 * V, V);
        check_launch();
      }
      T* fb = out->f_ext ? (T*)out->f_ext + (size_t)f * 3 * V : nullptr;
      for (int s = S - 1; s >= 0; --s) reverse_substep(c, D, fb, out->sphere, slot[f] * S + s, sv, f * S + s);
      HIPCHK(hipEventRecord(ev_rev[f], sv));
    }
    // the reverse stream waited for the last recomputation before frame 0
    HIPCHK(hipEventRecord(ev_end, sv));
    HIPCHK(hipStreamWaitEvent(st, ev_end, 0));
  }

  // adjoint state and gradient outputs before the first reversed frame:
  // FP64 accumulators of the per-constraint parameter gradients, sphere and
  // force gradients zeroed, xbar = 0, vbar = dL/dv_final
  static void begin_adjoint(xpbd_ctx c, int F, const void* dLdv, const xpbd_grads* out, hipStream_t st) {
    const int V = c->V;
    fill<double>(c->dist_acc, 0.0, c->n_dist, st);
    fill<double>(c->bend_acc, 0.0, c->n_bend, st);
    fill<double>(c->tet_acc, 0.0, (size_t)3 * c->n_tet, st);
    fill<double>(c->tri_acc, 0.0, (size_t)4 * c->n_tri, st);
    if (out->body_x) fill<double>(out->body_x, 0.0, (size_t)3 * c->body_nv, st);
    if (out->sphere) fill<double>(out->sphere, 0.0, 4, st);
    if (out->f_ext) fill<T>((T*)out->f_ext, T(0), (size_t)F * 3 * V, st);
    k_adj_init<T><<<nblocks(V), kBlock, 0, st>>>((V4*)c->XB, (V4*)c->VB, (const T*)c->w, (const T*)dLdv, V);
    check_launch();
  }

  // after the last reversed frame: dL/dx0, dL/dv0, and the parameter
  // gradients in the caller's constraint order
  static void finish_adjoint(xpbd_ctx c, const xpbd_params* p, const xpbd_grads* out, hipStream_t st) {
    const int V = c->V;
    if (out->x0) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->XB, (T*)out->x0, V);
    if (out->v0) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->VB, (T*)out->v0, V);
    check_launch();
    double ih2 = 1.0 / (c->h * c->h);
    if (out->dist_compliance && c->n_dist)
      k_scatter_alpha_grad<<<nblocks(c->n_dist), kBlock, 0, st>>>(c->dist_acc, c->dist_perm, out->dist_compliance,
                                                                  ih2, c->n_dist);
    if (out->bend_compliance && c->n_bend)
      k_scatter_alpha_grad<<<nblocks(c->n_bend), kBlock, 0, st>>>(c->bend_acc, c->bend_perm, out->bend_compliance,
                                                                  ih2, c->n_bend);
    if (out->tri_coef && c->n_tri)
      k_scatter_tri_grad<T><<<nblocks(c->n_tri), kBlock, 0, st>>>(c->tri_acc, c->tri_perm, (const T*)p->tri_coef,
                                                                  c->tri_area, out->tri_coef, ih2, c->n_tri);
    const bool want_E = out->tet_E && p->tet_E, want_lame = (out->tet_mu || out->tet_lambda) && p->tet_mu;
    if (c->n_mat && (want_E || want_lame)) {
      k_material_grad<T><<<c->n_mat, kBlock, 0, st>>>(
          c->tet_acc, c->mat_off, c->mat_items, want_E ? (const T*)p->tet_E : nullptr, (const T*)p->tet_mu,
          (const T*)p->tet_lambda, want_E ? out->tet_E : nullptr, want_lame ? out->tet_mu : nullptr,
          want_lame ? out->tet_lambda : nullptr, c->gamma_one, c->n_tet);
    } else if (c->n_tet) {
      if (want_E)
        k_scatter_E_grad<T><<<nblocks(c->n_tet), kBlock, 0, st>>>(c->tet_acc, c->tet_perm, (const T*)p->tet_E,
                                                                  out->tet_E, c->n_tet);
      if (want_lame)
        k_scatter_lame_grad<T><<<nblocks(c->n_tet), kBlock, 0, st>>>(c->tet_acc, c->tet_perm,
                                                                     (const T*)p->tet_mu, (const T*)p->tet_lambda,
                                                                     out->tet_mu, out->tet_lambda, c->gamma_one,
                                                                     c->n_tet);
    }
    check_launch();
  }

  static void ensure_parts(xpbd_ctx c, int F) {
    const size_t nb = nblocks((size_t)3 * c->V);
    if (c->parts_n < nb * F) {
      void* pp = c->parts;
      c->release(pp);
      c->parts = (double*)c->alloc(nb * F * sizeof(double));
      c->parts_n = nb * F;
    }
  }

  static void goal(xpbd_ctx c, const void* xf, const void* tg, const uint8_t* mask, const double* wv, int F,
                   double* loss, void* dLdx, hipStream_t st) {
    ensure_parts(c, F);
    goal_into(c, xf, tg, mask, wv, F, loss, dLdx, c->parts, st);
  }

  // parts: device [nblocks(3 V) * F] partial sums, each written before read
  static void goal_into(xpbd_ctx c, const void* xf, const void* tg, const uint8_t* mask, const double* wv, int F,
                        double* loss, void* dLdx, double* parts, hipStream_t st) {
    const size_t n = (size_t)3 * c->V;
    const size_t nb = nblocks(n);
    for (int f = 0; f < F; ++f) {
      int on = mask ? (mask[f] != 0) : 1;
      k_goal<T><<<nb, kBlock, 0, st>>>((const T*)xf + f * n, (const T*)tg + f * n, wv,
                                       dLdx ? (T*)dLdx + f * n : nullptr, n, on, parts + f * nb);
    }
    check_launch();
    if (loss) k_sum_parts<<<1, 1024, 0, st>>>(parts, nb * F, loss, 0);
    check_launch();
  }
};

// ===================================================================== create

template <class T>
void build_groups(xpbd_ctx c, const xpbd_schedule_desc* sd, const std::vector<int2>& didx,
                  const std::vector<double>& drest, const std::vector<int4>& bidx, const std::vector<double>& btheta,
                  const std::vector<int4>& tidx, const std::vector<double>& tB, const std::vector<int>& vid_c,
                  const std::vector<int4>& midx, const std::vector<double>& mB, const std::vector<int>& vid_bc);

void build(xpbd_ctx c, const xpbd_mesh_desc* m, const xpbd_constraint_desc* cd, const xpbd_schedule_desc* sd,
           const xpbd_options* o) {
  if (!m || !cd || !sd || !o) fail(XPBD_ERR_INVALID, "null descriptor");
  if (o->dtype != XPBD_F32 && o->dtype != XPBD_F64) fail(XPBD_ERR_INVALID, "bad dtype");
  if (!(o->dt > 0) || o->substeps < 1 || o->iterations < 0) fail(XPBD_ERR_INVALID, "bad dt/substeps/iterations");
  if (m->n_verts <= 0 || !m->rest_pos || !m->inv_mass) fail(XPBD_ERR_INVALID, "empty mesh");
  if (cd->n_dist < 0 || cd->n_bend < 0 || cd->n_tet < 0) fail(XPBD_ERR_INVALID, "negative counts");
  if ((cd->n_dist && !cd->dist_v) || (cd->n_bend && !cd->bend_v) || (cd->n_tet && (!cd->tet_v || !cd->tet_nu)))
    fail(XPBD_ERR_INVALID, "missing constraint arrays");
  if (o->tape_mode < 0 || o->tape_mode > 4) fail(XPBD_ERR_INVALID, "bad tape_mode");
  if (o->record_frames < 0) fail(XPBD_ERR_INVALID, "bad record_frames");
  if (o->launch_mode < 0 || o->launch_mode > 2 || o->persistent_blocks < 0)
    fail(XPBD_ERR_INVALID, "bad launch_mode / persistent_blocks");
  if (o->block_size != 0 &&
      (o->block_size < 64 || o->block_size > kMaxBlock || (o->block_size & (o->block_size - 1)) != 0))
    fail(XPBD_ERR_INVALID, "block_size must be 0 or a power of two in [64, %d]", kMaxBlock);
  c->block = o->block_size ? o->block_size : kBlock;
  if (o->group_records < 0 || o->group_records > 2) fail(XPBD_ERR_INVALID, "group_records must be 0, 1 or 2");
  if (o->group_block != 0 && (o->group_block < 64 || o->group_block > kBlock || (o->group_block & (o->group_block - 1))))
    fail(XPBD_ERR_INVALID, "group_block must be 0 or a power of two in [64, %d]", kBlock);
  c->group_stream = o->group_records == 2;
  c->group_block = o->group_block ? o->group_block : kBlock;
  if (o->record_kind < 0 || o->record_kind > 1) fail(XPBD_ERR_INVALID, "record_kind must be 0 or 1");
  if (o->record_kind == 1 && o->launch_mode == 2)
    fail(XPBD_ERR_INVALID, "record_kind 1 needs LDS group launches, not the persistent kernel");
  c->record_kind = o->record_kind;
  c->dtype = o->dtype;
  c->tsz = o->dtype == XPBD_F32 ? 4 : 8;
  c->V = m->n_verts;
  c->n_dist = cd->n_dist;
  c->n_bend = cd->n_bend;
  c->n_tet = cd->n_tet;
  c->dt = o->dt;
  c->S = o->substeps;
  c->K = o->iterations;
  c->h = o->dt / o->substeps;
  for (int a = 0; a < 3; ++a) c->g[a] = o->gravity[a];
  c->budget = o->hbm_budget_bytes;
  c->gamma_one = o->tet_gamma_one ? 1 : 0;
  c->tape_mode_opt = o->tape_mode;
  c->record_frames_opt = o->record_frames;
  c->serial_adjoint = o->serial_adjoint ? 1 : 0;
  c->tau = cd->contact_thickness;
  c->alpha_c = cd->contact_compliance;
  const int V = c->V;
  for (int k = 0; k < V; ++k) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(m->rest_pos[3 * k + a])) fail(XPBD_ERR_INVALID, "rest position %d not finite", k);
    if (!(m->inv_mass[k] >= 0) || !std::isfinite(m->inv_mass[k])) fail(XPBD_ERR_INVALID, "bad inverse mass at %d", k);
  }
  auto check_idx = [&](const int32_t* v, int n, int k, const char* what) {
    for (int64_t i = 0; i < (int64_t)n * k; ++i)
      if (v[i] < 0 || v[i] >= V) fail(XPBD_ERR_INVALID, "%s index out of range", what);
  };
  check_idx(cd->dist_v, cd->n_dist, 2, "distance");
  check_idx(cd->bend_v, cd->n_bend, 4, "bending");
  check_idx(cd->tet_v, cd->n_tet, 4, "tet");
  for (int t = 0; t < cd->n_tet; ++t)
    if (!(cd->tet_nu[t] > -1.0 && cd->tet_nu[t] < 0.5)) fail(XPBD_ERR_INVALID, "Poisson ratio of tet %d out of range", t);
  if (cd->n_tri < 0 || (cd->n_tri > 0 && (!cd->tri_v || !cd->tri_uv))) fail(XPBD_ERR_INVALID, "bad membrane arrays");
  c->n_tri = cd->n_tri;
  check_idx(cd->tri_v, cd->n_tri, 3, "membrane");
  for (int64_t i = 0; i < 6 * (int64_t)cd->n_tri; ++i)
    if (!std::isfinite(cd->tri_uv[i])) fail(XPBD_ERR_INVALID, "membrane material coordinates not finite");
  if (cd->n_body_tris < 0 || cd->n_body_verts < 0 || (cd->n_body_tris > 0 && !cd->body_tris))
    fail(XPBD_ERR_INVALID, "bad body collider arrays");
  c->body_nv = cd->n_body_verts;
  c->body_nt = cd->n_body_tris;
  for (int64_t i = 0; i < 3 * (int64_t)cd->n_body_tris; ++i)
    if (cd->body_tris[i] < 0 || cd->body_tris[i] >= cd->n_body_verts) fail(XPBD_ERR_INVALID, "body triangle index out of range");
  if (cd->n_body_tris > 0 &&
      (!(cd->body_radius > 0) || !std::isfinite(cd->body_radius) || !std::isfinite(cd->body_thickness) ||
       !(cd->body_compliance >= 0) || !std::isfinite(cd->body_compliance)))
    fail(XPBD_ERR_INVALID, "body collider: radius > 0, finite thickness and compliance >= 0 required");
  c->b_tau = cd->body_thickness;
  c->b_alpha = cd->body_compliance;
  c->b_radius = cd->body_radius;
  c->body_tris_h.assign(cd->body_tris, cd->body_tris + 3 * (int64_t)std::max(cd->n_body_tris, 0));
  if (cd->n_materials < 0 || (cd->n_materials > 0 && cd->n_tet > 0 && !cd->tet_material))
    fail(XPBD_ERR_INVALID, "bad material clusters");
  c->n_mat = cd->n_materials;
  for (int t = 0; c->n_mat && t < cd->n_tet; ++t)
    if (cd->tet_material[t] < 0 || cd->tet_material[t] >= c->n_mat)
      fail(XPBD_ERR_INVALID, "material of tet %d out of range", t);

  // ---- schedule: validate, then lay out internal order set by set
  if (sd->n_sets < 0 || (sd->n_sets > 0 && (!sd->set_type || !sd->set_offsets || !sd->set_items)))
    fail(XPBD_ERR_INVALID, "bad schedule");
  std::vector<int> seen_d(c->n_dist, 0), seen_b(c->n_bend, 0), seen_t(c->n_tet, 0), seen_c(V, 0);
  std::vector<int> seen_m(c->n_tri, 0), seen_bc(V, 0);
  std::vector<int> stamp(V, -1);
  std::vector<int> perm_d, perm_b, perm_t, vid_c, perm_m, vid_bc;
  perm_d.reserve(c->n_dist);
  perm_b.reserve(c->n_bend);
  perm_t.reserve(c->n_tet);
  if (sd->n_sets > 0 && sd->set_offsets[0] != 0) fail(XPBD_ERR_INVALID, "set_offsets[0] must be 0");
  // LDS groups: which group each set belongs to
  std::vector<int> set_group(std::max(sd->n_sets, 0), -1);
  if (sd->n_groups < 0 || (sd->n_groups > 0 && (!sd->group_sets || !sd->group_patch)))
    fail(XPBD_ERR_INVALID, "bad group arrays");
  for (int g = 0; g < sd->n_groups; ++g) {
    int a = sd->group_sets[2 * g], b = sd->group_sets[2 * g + 1];
    if (a < 0 || b > sd->n_sets || b <= a || b - a > kMaxGroupSets)
      fail(XPBD_ERR_INVALID, "group %d: bad set range [%d, %d)", g, a, b);
    for (int q = a; q < b; ++q) {
      if (set_group[q] >= 0) fail(XPBD_ERR_INVALID, "groups %d and %d overlap", set_group[q], g);
      set_group[q] = g;
    }
    for (int v = 0; v < V; ++v)
      if (sd->group_patch[(size_t)g * V + v] < 0) fail(XPBD_ERR_INVALID, "group %d: negative patch id", g);
  }
  for (int s = 0; s < sd->n_sets; ++s) {
    int ty = sd->set_type[s];
    int64_t b = sd->set_offsets[s], e = sd->set_offsets[s + 1];
    if (e < b) fail(XPBD_ERR_INVALID, "set %d: decreasing offsets", s);
    if (ty < 0 || ty > 5) fail(XPBD_ERR_INVALID, "set %d: bad type", s);
    if (ty == XPBD_BODY && c->body_nt == 0) fail(XPBD_ERR_INVALID, "set %d: body-contact set without a body", s);
    if (ty == XPBD_CONTACT && !cd->contact) fail(XPBD_ERR_INVALID, "set %d: contact set but contact disabled", s);
    // order items inside the set by patch (grouped sets), then by their
    // smallest vertex (locality)
    const int32_t* gpatch = set_group[s] >= 0 ? sd->group_patch + (size_t)set_group[s] * V : nullptr;
    std::vector<std::pair<int64_t, int>> items;
    items.reserve(e - b);
    for (int64_t q = b; q < e; ++q) {
      int it = sd->set_items[q];
      const int32_t* vv = nullptr;
      int nv = 1, lim = V;
      if (ty == XPBD_DIST) { lim = c->n_dist; nv = 2; }
      else if (ty == XPBD_BEND) { lim = c->n_bend; nv = 4; }
      else if (ty == XPBD_TET) { lim = c->n_tet; nv = 4; }
      else if (ty == XPBD_TRI) { lim = c->n_tri; nv = 3; }
      if (it < 0 || it >= lim) fail(XPBD_ERR_INVALID, "set %d: item %d out of range", s, it);
      if (ty == XPBD_DIST) vv = cd->dist_v + 2 * (int64_t)it;
      else if (ty == XPBD_BEND) vv = cd->bend_v + 4 * (int64_t)it;
      else if (ty == XPBD_TET) vv = cd->tet_v + 4 * (int64_t)it;
      else if (ty == XPBD_TRI) vv = cd->tri_v + 3 * (int64_t)it;
      int key = INT32_MAX;
      int64_t patch = 0;
      for (int k = 0; k < nv; ++k) {
        int v = vv ? vv[k] : it;
        if (stamp[v] == s) fail(XPBD_ERR_INVALID, "set %d is not independent: vertex %d appears twice", s, v);
        stamp[v] = s;
        key = std::min(key, v);
        if (gpatch) {
          if (k == 0) patch = gpatch[v];
          else if (gpatch[v] != patch)
            fail(XPBD_ERR_INVALID, "set %d (group %d): a constraint spans two patches", s, set_group[s]);
        }
      }
      int* seen = ty == XPBD_DIST ? &seen_d[it] : ty == XPBD_BEND ? &seen_b[it] : ty == XPBD_TET ? &seen_t[it]
                : ty == XPBD_TRI ? &seen_m[it] : ty == XPBD_BODY ? &seen_bc[it] : &seen_c[it];
      if (*seen) fail(XPBD_ERR_INVALID, "constraint %d of type %d appears twice in the schedule", it, ty);
      *seen = 1;
      if ((ty == XPBD_CONTACT || ty == XPBD_BODY) && !(m->inv_mass[it] > 0))
        fail(XPBD_ERR_INVALID, "contact on pinned vertex %d", it);
      items.push_back({(patch << 32) | (int64_t)key, it});
    }
    std::stable_sort(items.begin(), items.end());
    SetInfo si{};
    si.type = ty;
    si.count = (int)items.size();
    std::vector<int>& dst = ty == XPBD_DIST ? perm_d : ty == XPBD_BEND ? perm_b : ty == XPBD_TET ? perm_t
                          : ty == XPBD_TRI ? perm_m : ty == XPBD_BODY ? vid_bc : vid_c;
    si.begin = (int)dst.size();
    for (auto& pr : items) dst.push_back(pr.second);
    c->sets.push_back(si);
  }
  for (int i = 0; i < c->n_dist; ++i) if (!seen_d[i]) fail(XPBD_ERR_INVALID, "distance constraint %d not scheduled", i);
  for (int i = 0; i < c->n_bend; ++i) if (!seen_b[i]) fail(XPBD_ERR_INVALID, "bending constraint %d not scheduled", i);
  for (int i = 0; i < c->n_tet; ++i) if (!seen_t[i]) fail(XPBD_ERR_INVALID, "tet %d not scheduled", i);
  for (int i = 0; i < c->n_tri; ++i) if (!seen_m[i]) fail(XPBD_ERR_INVALID, "membrane triangle %d not scheduled", i);
  c->n_contact = (int)vid_c.size();
  c->n_bc = (int)vid_bc.size();
  // per-iteration record layout
  size_t off = 0;
  for (SetInfo& si : c->sets) {
    si.tape_off = off;
    off += align256(tape_item_bytes(si.type, c->tsz) * (size_t)si.count);
    c->proj_per_iter += si.type == XPBD_TET ? 2 * (int64_t)si.count : si.count;
  }
  c->iter_tape_bytes = off;

  // ---- rest data in internal order (FP64 on the host)
  std::vector<int2> didx(c->n_dist);
  std::vector<double> drest(c->n_dist);
  for (int i = 0; i < c->n_dist; ++i) {
    int u = perm_d[i];
    int a = cd->dist_v[2 * u], b = cd->dist_v[2 * u + 1];
    H3 r = hsub(hv(m->rest_pos, a), hv(m->rest_pos, b));
    double L = std::sqrt(hdot(r, r));
    if (!(L > 0)) fail(XPBD_ERR_INVALID, "distance constraint %d has zero rest length", u);
    didx[i] = make_int2(a, b);
    drest[i] = L;
  }
  std::vector<int4> bidx(c->n_bend);
  std::vector<double> btheta(c->n_bend);
  for (int i = 0; i < c->n_bend; ++i) {
    int u = perm_b[i];
    const int32_t* q = cd->bend_v + 4 * (int64_t)u;
    double th;
    if (!rest_dihedral(hv(m->rest_pos, q[0]), hv(m->rest_pos, q[1]), hv(m->rest_pos, q[2]), hv(m->rest_pos, q[3]), &th))
      fail(XPBD_ERR_INVALID, "bending constraint %d has a degenerate rest hinge", u);
    bidx[i] = make_int4(q[0], q[1], q[2], q[3]);
    btheta[i] = th;
  }
  std::vector<int4> tidx(c->n_tet);
  std::vector<double> tB((size_t)9 * c->n_tet), tvol(c->n_tet), tnu(c->n_tet);
  for (int i = 0; i < c->n_tet; ++i) {
    int u = perm_t[i];
    const int32_t* q = cd->tet_v + 4 * (int64_t)u;
    double B[9], vol;
    if (!rest_tet(hv(m->rest_pos, q[0]), hv(m->rest_pos, q[1]), hv(m->rest_pos, q[2]), hv(m->rest_pos, q[3]), B, &vol))
      fail(XPBD_ERR_INVALID, "tet %d has non-positive rest volume", u);
    tidx[i] = make_int4(q[0], q[1], q[2], q[3]);
    for (int r = 0; r < 9; ++r) tB[(size_t)r * c->n_tet + i] = B[r];
    tvol[i] = vol;
    tnu[i] = cd->tet_nu[u];
  }

  // membrane: Dm^-1 from the material-space (u, v) corners, area |det Dm| / 2
  std::vector<int4> midx(c->n_tri);
  std::vector<double> mB((size_t)4 * c->n_tri), marea(c->n_tri);
  for (int i = 0; i < c->n_tri; ++i) {
    int u = perm_m[i];
    const int32_t* q = cd->tri_v + 3 * (int64_t)u;
    const double* uv = cd->tri_uv + 6 * (int64_t)u;
    double a = uv[2] - uv[0], b = uv[4] - uv[0], cc = uv[3] - uv[1], d = uv[5] - uv[1];
    double det = a * d - b * cc;
    if (!(std::fabs(det) > 0)) fail(XPBD_ERR_INVALID, "membrane triangle %d has zero material-space area", u);
    midx[i] = make_int4(q[0], q[1], q[2], 0);
    mB[i] = d / det;
    mB[(size_t)c->n_tri + i] = -b / det;
    mB[2 * (size_t)c->n_tri + i] = -cc / det;
    mB[3 * (size_t)c->n_tri + i] = a / det;
    marea[i] = 0.5 * std::fabs(det);
  }

  // ---- device allocations
  const size_t T_ = c->tsz;
  const size_t V4b = 4 * T_;
  c->w = c->alloc(V * T_);
  c->dev_blk = c->alloc(2 * kDevBlk);
  c->X = c->alloc(V * V4b);
  c->Vv = c->alloc(V * V4b);
  c->Xp = c->alloc(V * V4b);
  c->flag = (int*)c->alloc(sizeof(int));
  c->bar = (unsigned*)c->alloc(((size_t)4096 * kFlagStride + 1) * sizeof(unsigned));
  c->abort_flag = (int*)c->alloc(sizeof(int));
  HIPCHK(hipMemset(c->abort_flag, 0, sizeof(int)));
  std::vector<double> wv(m->inv_mass, m->inv_mass + V);
  auto up_T = [&](void* dst, const std::vector<double>& v) {
    if (c->dtype == XPBD_F32) c->upload(dst, cast_vec<float>(v));
    else c->upload(dst, v);
  };
  up_T(c->w, wv);
  if (c->n_dist) {
    int n = c->n_dist;
    c->dist_idx = (int2*)c->alloc(n * sizeof(int2));
    c->dist_rest = c->alloc(n * T_);
    c->dist_perm = (int*)c->alloc(n * sizeof(int));
    c->dist_at = c->alloc(n * T_);
    c->dist_lam = c->alloc(n * T_);
    c->upload(c->dist_idx, didx);
    up_T(c->dist_rest, drest);
    c->upload(c->dist_perm, perm_d);
  }
  if (c->n_bend) {
    int n = c->n_bend;
    c->bend_idx = (int4*)c->alloc(n * sizeof(int4));
    c->bend_theta0 = c->alloc(n * T_);
    c->bend_perm = (int*)c->alloc(n * sizeof(int));
    c->bend_at = c->alloc(n * T_);
    c->bend_lam = c->alloc(n * T_);
    c->upload(c->bend_idx, bidx);
    up_T(c->bend_theta0, btheta);
    c->upload(c->bend_perm, perm_b);
  }
  if (c->n_tet) {
    int n = c->n_tet;
    c->tet_idx = (int4*)c->alloc(n * sizeof(int4));
    c->tet_B = c->alloc((size_t)9 * n * T_);
    c->tet_perm = (int*)c->alloc(n * sizeof(int));
    c->tet_nu = (double*)c->alloc(n * sizeof(double));
    c->tet_vol = (double*)c->alloc(n * sizeof(double));
    c->tet_atD = c->alloc(n * T_);
    c->tet_atH = c->alloc(n * T_);
    c->tet_gamma = c->alloc(n * T_);
    c->tet_lamD = c->alloc(n * T_);
    c->tet_lamH = c->alloc(n * T_);
    c->upload(c->tet_idx, tidx);
    up_T(c->tet_B, tB);
    c->upload(c->tet_perm, perm_t);
    c->upload(c->tet_nu, tnu);
    c->upload(c->tet_vol, tvol);
    if (c->n_mat) {
      std::vector<int> pidx(n), moff(c->n_mat + 1, 0), mitems(n);
      for (int i = 0; i < n; ++i) ++moff[(pidx[i] = cd->tet_material[perm_t[i]]) + 1];
      for (int q = 0; q < c->n_mat; ++q) moff[q + 1] += moff[q];
      std::vector<int> fillp(moff.begin(), moff.end() - 1);
      for (int i = 0; i < n; ++i) mitems[fillp[pidx[i]]++] = i;
      c->tet_pidx = (int*)c->alloc(n * sizeof(int));
      c->mat_off = (int*)c->alloc((c->n_mat + 1) * sizeof(int));
      c->mat_items = (int*)c->alloc(n * sizeof(int));
      c->upload(c->tet_pidx, pidx);
      c->upload(c->mat_off, moff);
      c->upload(c->mat_items, mitems);
    } else {
      c->tet_pidx = c->tet_perm;
    }
  }
  if (c->n_tri) {
    int n = c->n_tri;
    c->tri_idx = (int4*)c->alloc(n * sizeof(int4));
    c->tri_B = c->alloc((size_t)4 * n * T_);
    c->tri_perm = (int*)c->alloc(n * sizeof(int));
    c->tri_area = (double*)c->alloc(n * sizeof(double));
    c->tri_at = c->alloc((size_t)4 * n * T_);
    c->tri_lam = c->alloc((size_t)3 * n * T_);
    c->upload(c->tri_idx, midx);
    up_T(c->tri_B, mB);
    c->upload(c->tri_perm, perm_m);
    c->upload(c->tri_area, marea);
  }
  if (c->body_nt) {
    std::vector<int4> bt(c->body_nt);
    for (int t = 0; t < c->body_nt; ++t)
      bt[t] = make_int4(cd->body_tris[3 * t], cd->body_tris[3 * t + 1], cd->body_tris[3 * t + 2], 0);
    c->body_tris = (int4*)c->alloc(c->body_nt * sizeof(int4));
    c->upload(c->body_tris, bt);
  }
  if (c->n_bc) {
    c->bc_vid = (int*)c->alloc(c->n_bc * sizeof(int));
    c->bc_lam = c->alloc(c->n_bc * T_);
    c->upload(c->bc_vid, vid_bc);
  }
  if (c->n_contact) {
    int n = c->n_contact;
    c->contact_vid = (int*)c->alloc(n * sizeof(int));
    c->contact_lam = c->alloc(n * T_);
    c->upload(c->contact_vid, vid_c);
    std::vector<int> order(n);
    for (const SetInfo& si : c->sets) {
      if (si.type != XPBD_CONTACT) continue;
      std::vector<int> loc(si.count);
      for (int i = 0; i < si.count; ++i) loc[i] = i;
      std::sort(loc.begin(), loc.end(), [&](int x, int y) { return vid_c[si.begin + x] < vid_c[si.begin + y]; });
      for (int i = 0; i < si.count; ++i) order[si.begin + i] = loc[i];
    }
    c->contact_order = (int*)c->alloc(n * sizeof(int));
    c->upload(c->contact_order, order);
  }

  // ---- LDS groups
  c->group_at_start.assign(c->sets.size(), -1);
  c->group_at_end.assign(c->sets.size(), -1);
  if (sd->n_groups > 0 && o->launch_mode != 2) {
    if (c->dtype == XPBD_F32) build_groups<float>(c, sd, didx, drest, bidx, btheta, tidx, tB, vid_c, midx, mB, vid_bc);
    else build_groups<double>(c, sd, didx, drest, bidx, btheta, tidx, tB, vid_c, midx, mB, vid_bc);
  } else {
    for (int g = 0; g < sd->n_groups; ++g) {
      xpbd_ctx_s::Group G;
      G.a = sd->group_sets[2 * g];
      G.b = sd->group_sets[2 * g + 1];
      c->groups.push_back(G);
    }
  }
  // per-iteration record layout: sets outside LDS groups, then one chunk per LDS group
  size_t toff = 0;
  for (size_t k = 0; k < c->sets.size(); ++k) {
    SetInfo& si = c->sets[k];
    int g = -1;
    for (size_t q = 0; q < c->groups.size(); ++q)
      if (c->groups[q].lds && (int)k >= c->groups[q].a && (int)k < c->groups[q].b) g = (int)q;
    if (g >= 0) continue;
    si.tape_off = toff;
    toff += align256(tape_item_bytes(si.type, c->tsz) * (size_t)si.count);
  }
  for (auto& G : c->groups)
    if (G.lds) {
      G.tape_off = (long long)toff;
      toff += align256(G.tape_bytes);
    }
  c->iter_tape_bytes = toff;
  if (c->record_kind == 1) {
    // snapshots instead: every set must run inside an LDS group launch
    for (size_t k = 0; k < c->sets.size(); ++k) {
      bool in = false;
      for (const auto& G : c->groups) in = in || (G.lds && (int)k >= G.a && (int)k < G.b);
      if (!in) fail(XPBD_ERR_INVALID, "record_kind 1: set %zu does not run in an LDS group", k);
    }
    size_t so = 0, scr = 0;
    for (auto& G : c->groups) {
      if (!G.lds) continue;
      // entries streamed: the replayed record goes to LDS when the patch's
      // record and its two tiles fit in 64 KB (several workgroups per CU),
      // else to a scratch buffer in global memory
      G.replay_lds = c->group_stream && 2 * G.smem_tile + G.max_tbytes <= 65536;
      const size_t extra = c->group_stream ? 2 * G.smem_tile + (G.replay_lds ? G.max_tbytes : 0)
                                           : G.smem_rev + G.smem_tile;
      if (extra > c->lds_limit) fail(XPBD_ERR_INVALID, "record_kind 1: a patch's replay needs %zu bytes of LDS", extra);
      G.snap_x_off = (long long)so;
      so += align256(3 * c->tsz * G.n_staged);
      G.snap_l_off = (long long)so;
      so += align256(G.fmul_bytes);
      if (c->group_stream && !G.replay_lds) scr = std::max(scr, G.tape_bytes);
      c->max_group_lds = std::max(c->max_group_lds, (int)extra);
    }
    c->iter_tape_bytes = so;
    c->scratch_bytes = c->group_stream ? scr : 0;
    if (c->dtype == XPBD_F32) Ops<float>::allow_lds((size_t)c->max_group_lds);
    else Ops<double>::allow_lds((size_t)c->max_group_lds);
  }
}

// Build the LDS launch data of every schedule group: patch vertex lists,
// per-patch item counts, the constant entry image in its LDS layout (static
// fields here; compliances are filled per call) and the offsets of the
// forward and reverse state images.
template <class T>
void build_groups(xpbd_ctx c, const xpbd_schedule_desc* sd, const std::vector<int2>& didx,
                  const std::vector<double>& drest, const std::vector<int4>& bidx, const std::vector<double>& btheta,
                  const std::vector<int4>& tidx, const std::vector<double>& tB, const std::vector<int>& vid_c,
                  const std::vector<int4>& midx, const std::vector<double>& mB, const std::vector<int>& vid_bc) {
  const int V = c->V;
  {
    int dev = 0, lim = 0, optin = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) {
      (void)hipGetLastError();
      optin = 0;
    }
    c->lds_limit = (size_t)std::max(lim, optin);
  }
  auto verts_of = [&](int type, int j, int out[4]) -> int {
    switch (type) {
      case XPBD_DIST: out[0] = didx[j].x; out[1] = didx[j].y; return 2;
      case XPBD_BEND: out[0] = bidx[j].x; out[1] = bidx[j].y; out[2] = bidx[j].z; out[3] = bidx[j].w; return 4;
      case XPBD_TET: out[0] = tidx[j].x; out[1] = tidx[j].y; out[2] = tidx[j].z; out[3] = tidx[j].w; return 4;
      case XPBD_TRI: out[0] = midx[j].x; out[1] = midx[j].y; out[2] = midx[j].z; return 3;
      case XPBD_BODY: out[0] = vid_bc[j]; return 1;
      default: out[0] = vid_c[j]; return 1;
    }
  };
  // entry positions per constraint for the per-call compliance fill:
  // distance, bending, tet, membrane
  const int ntype[4] = {c->n_dist, c->n_bend, c->n_tet, c->n_tri};
  std::vector<long long> gpos[4];
  for (int t = 0; t < 4; ++t) gpos[t].assign(ntype[t], -1);
  std::vector<unsigned char> img;          // constant entries of every LDS group
  size_t fmul_total = 0, rmul_total = 0;   // bytes of the two state images
  std::vector<int> lidx(V, -1);
  std::vector<char> ref(V, 0);
  for (int g = 0; g < sd->n_groups; ++g) {
    xpbd_ctx_s::Group G;
    G.a = sd->group_sets[2 * g];
    G.b = sd->group_sets[2 * g + 1];
    const int ns = G.b - G.a;
    const int32_t* gp = sd->group_patch + (size_t)g * V;
    std::fill(ref.begin(), ref.end(), 0);
    for (int q = G.a; q < G.b; ++q) {
      const SetInfo& si = c->sets[q];
      for (int i = 0; i < si.count; ++i) {
        int vv[4];
        int nv = verts_of(si.type, si.begin + i, vv);
        for (int k = 0; k < nv; ++k) ref[vv[k]] = 1;
      }
      G.items += si.type == XPBD_TET ? 2 * (int64_t)si.count : si.count;
      if (si.type == XPBD_TET || si.type == XPBD_TRI || si.type == XPBD_BODY) G.heavy = true;
    }
    std::vector<int> raw;
    for (int v = 0; v < V; ++v) if (ref[v]) raw.push_back(gp[v]);
    std::sort(raw.begin(), raw.end());
    raw.erase(std::unique(raw.begin(), raw.end()), raw.end());
    const int P = (int)raw.size();
    G.P = P;
    auto cpatch = [&](int v) { return (int)(std::lower_bound(raw.begin(), raw.end(), gp[v]) - raw.begin()); };
    std::vector<int> pv_start(P + 1, 0), pv;
    for (int v = 0; v < V; ++v) if (ref[v]) pv_start[cpatch(v) + 1]++;
    for (int p = 0; p < P; ++p) pv_start[p + 1] += pv_start[p];
    pv.resize(pv_start[P]);
    {
      std::vector<int> fillp(pv_start.begin(), pv_start.end() - 1);
      for (int v = 0; v < V; ++v)
        if (ref[v]) {
          int cp = cpatch(v);
          lidx[v] = fillp[cp] - pv_start[cp];
          pv[fillp[cp]++] = v;
        }
    }
    int nv_max = 0;
    for (int p = 0; p < P; ++p) nv_max = std::max(nv_max, pv_start[p + 1] - pv_start[p]);
    // items of each set per patch (items are sorted by patch inside a set)
    std::vector<int> cnt((size_t)P * ns, 0), first((size_t)P * ns, 0), stype(ns);
    for (int q = 0; q < ns; ++q) {
      const SetInfo& si = c->sets[G.a + q];
      stype[q] = si.type;
      for (int i = 0; i < si.count; ++i) {
        int vv[4];
        verts_of(si.type, si.begin + i, vv);
        cnt[(size_t)cpatch(vv[0]) * ns + q]++;
      }
      int acc = si.begin;
      for (int p = 0; p < P; ++p) {
        first[(size_t)p * ns + q] = acc;
        acc += cnt[(size_t)p * ns + q];
      }
    }
    // sizes per patch
    std::vector<long long> ioff(P), fmoff(P), rmoff(P), tpos(P);
    size_t mf = 0, mr = 0, isum = 0, fmsum = 0, rmsum = 0, tsum = 0;
    for (int p = 0; p < P; ++p) {
      size_t vb = al32((size_t)(pv_start[p + 1] - pv_start[p]) * sizeof(Vec4<T>));
      size_t ib = 0, fb = 0, rb = 0, tb = 0;  // entries, forward state, reverse state, record
      for (int q = 0; q < ns; ++q) {
        size_t n = cnt[(size_t)p * ns + q];
        ib += al32(n * rec_bytes<T>(stype[q]));
        fb += al32(n * fmul_words(stype[q]) * sizeof(T));
        rb += al32(n * rmul_words(stype[q]) * sizeof(T));
        tb += al32(n * tape_words(stype[q]) * sizeof(T));
      }
      ioff[p] = (long long)(img.size() + isum);
      fmoff[p] = (long long)(fmul_total + fmsum);
      rmoff[p] = (long long)(rmul_total + rmsum);
      tpos[p] = (long long)tsum;
      isum += ib; fmsum += fb; rmsum += rb; tsum += tb;
      mf = std::max(mf, vb + ib + fb);
      mr = std::max(mr, vb + ib + rb + tb);
      G.max_tbytes = std::max(G.max_tbytes, tb);
    }
    G.smem_fwd = mf;
    G.smem_rev = mr;
    G.smem_tile = al32((size_t)nv_max * sizeof(Vec4<T>));
    G.tape_bytes = tsum;
    G.n_staged = (size_t)pv_start[P];
    G.fmul_lo = (long long)fmul_total;
    G.fmul_bytes = fmsum;
    G.lds = P > 0 && nv_max <= 65535 && (c->group_stream ? G.smem_tile : std::max(mf, mr)) <= c->lds_limit;
    if (G.lds) {
      // constant entries in LDS layout; the state images are zeroed on the device
      img.resize(img.size() + isum, 0);
      fmul_total += fmsum;
      rmul_total += rmsum;
      for (int p = 0; p < P; ++p) {
        size_t io = (size_t)ioff[p];
        for (int q = 0; q < ns; ++q) {
          const int n = cnt[(size_t)p * ns + q], ty = stype[q];
          for (int i = 0; i < n; ++i) {
            int j = first[(size_t)p * ns + q] + i;
            int vv[4] = {0, 0, 0, 0};
            int nv = verts_of(ty, j, vv);
            unsigned l[4] = {0, 0, 0, 0};
            for (int k = 0; k < nv; ++k) l[k] = (unsigned)lidx[vv[k]];
            unsigned l01 = l[0] | (l[1] << 16), l23 = l[2] | (l[3] << 16);
            unsigned char* ip = &img[io + i * rec_bytes<T>(ty)];
            switch (ty) {
              case XPBD_DIST: {
                SDist<T> e{(T)drest[j], T(0), l01};
                std::memcpy(ip, &e, sizeof e);
                break;
              }
              case XPBD_BEND: {
                SBend<T> e{(T)btheta[j], T(0), l01, l23};
                std::memcpy(ip, &e, sizeof e);
                break;
              }
              case XPBD_TET: {
                STet<T> e{};
                for (int k = 0; k < 9; ++k) e.B[k] = (T)tB[(size_t)k * c->n_tet + j];
                e.l01 = l01;
                e.l23 = l23;
                std::memcpy(ip, &e, sizeof e);
                break;
              }
              case XPBD_BODY: {
                SBody<T> e{l[0], j};
                std::memcpy(ip, &e, sizeof e);
                break;
              }
              case XPBD_TRI: {
                STri<T> e{};
                for (int k = 0; k < 4; ++k) e.B[k] = (T)mB[(size_t)k * c->n_tri + j];
                e.l01 = l01;
                e.l2 = l[2];
                std::memcpy(ip, &e, sizeof e);
                break;
              }
              default: {
                SCon<T> e{l[0]};
                std::memcpy(ip, &e, sizeof e);
                break;
              }
            }
            if (ty != XPBD_CONTACT && ty != XPBD_BODY)
              gpos[ty == XPBD_TRI ? 3 : ty][j] = (long long)(io + i * rec_bytes<T>(ty));
          }
          io += al32((size_t)n * rec_bytes<T>(ty));
        }
      }
      c->max_group_lds = std::max(c->max_group_lds, (int)(c->group_stream ? G.smem_tile : std::max(mf, mr)));
      G.pv_start = (int*)c->alloc(pv_start.size() * sizeof(int));
      G.pv = (int*)c->alloc(pv.size() * sizeof(int));
      G.cnt = (int*)c->alloc(cnt.size() * sizeof(int));
      G.rec_first = (int*)c->alloc(first.size() * sizeof(int));
      G.set_type = (int*)c->alloc(ns * sizeof(int));
      G.img = (long long*)c->alloc(P * sizeof(long long));
      G.fmul = (long long*)c->alloc(P * sizeof(long long));
      G.rmul = (long long*)c->alloc(P * sizeof(long long));
      G.tpos = (long long*)c->alloc(P * sizeof(long long));
      c->upload(G.pv_start, pv_start);
      c->upload(G.pv, pv);
      c->upload(G.cnt, cnt);
      c->upload(G.rec_first, first);
      c->upload(G.set_type, stype);
      c->upload(G.img, ioff);
      c->upload(G.fmul, fmoff);
      c->upload(G.rmul, rmoff);
      c->upload(G.tpos, tpos);
      c->group_at_start[G.a] = g;
      c->group_at_end[G.b - 1] = g;
    }
    c->groups.push_back(G);
  }
  if (!img.empty()) {
    c->gimg = (char*)c->alloc(img.size());
    c->upload(c->gimg, img);
    c->gfmul = (char*)c->alloc(fmul_total);
    c->grmul = (char*)c->alloc(rmul_total);
    HIPCHK(hipMemset(c->gfmul, 0, fmul_total));
    HIPCHK(hipMemset(c->grmul, 0, rmul_total));
    for (int t = 0; t < 4; ++t)
      if (ntype[t]) {
        c->gpos[t] = (long long*)c->alloc(ntype[t] * sizeof(long long));
        c->upload(c->gpos[t], gpos[t]);
      }
    Ops<T>::allow_lds((size_t)c->max_group_lds);
  }
}

// plain launches or the persistent program kernel
void choose_launch(xpbd_ctx c, const xpbd_options* o) {
  c->prog_blocks_opt = o->persistent_blocks;
  if (o->launch_mode == 1) { c->persistent = false; return; }
  int dev = 0, coop = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (o->launch_mode == 2) {
    if (!coop) fail(XPBD_ERR_INVALID, "launch_mode 2 needs cooperative launch support");
    if (c->n_bc) fail(XPBD_ERR_INVALID, "launch_mode 2 does not run body-contact sets (per-substep pairing)");
    c->persistent = true;
    return;
  }
  // auto: one launch per set.  Measured on MI355X (cloth 256x256, sets of
  // 12k-65k constraints): a launch costs about 4.3 us, while a grid-wide
  // barrier across the 8 XCDs costs 7-16 us (each block's agent-scope fences
  // write back and invalidate its XCD's L2), so the persistent kernel is
  // only used when asked for.
  c->persistent = false;
  (void)coop;
}

// allocate the adjoint working set for a tape of `slots` substeps
void ensure_adjoint_buffers(xpbd_ctx c, int slots) {
  const size_t T_ = c->tsz, V4b = 4 * T_;
  if (!c->XB) {
    c->XB = c->alloc(c->V * V4b);
    c->VB = c->alloc(c->V * V4b);
    if (c->n_dist) {
      c->dist_lamb = c->alloc(c->n_dist * T_);
      c->dist_ab = c->alloc(c->n_dist * T_);
      c->dist_acc = (double*)c->alloc(c->n_dist * sizeof(double));
    }
    if (c->n_bend) {
      c->bend_lamb = c->alloc(c->n_bend * T_);
      c->bend_ab = c->alloc(c->n_bend * T_);
      c->bend_acc = (double*)c->alloc(c->n_bend * sizeof(double));
    }
    if (c->n_tet) {
      c->tet_lambD = c->alloc(c->n_tet * T_);
      c->tet_lambH = c->alloc(c->n_tet * T_);
      c->tet_eb = c->alloc(3 * c->n_tet * T_);
      c->tet_acc = (double*)c->alloc(3 * c->n_tet * sizeof(double));
    }
    if (c->n_contact) {
      c->contact_lamb = c->alloc(c->n_contact * T_);
      c->contact_sacc = c->alloc(c->n_contact * V4b);
    }
    if (c->n_bc) c->bc_lamb = c->alloc(c->n_bc * T_);
    if (c->n_tri) {
      c->tri_lamb = c->alloc((size_t)3 * c->n_tri * T_);
      c->tri_ab = c->alloc((size_t)4 * c->n_tri * T_);
      c->tri_acc = (double*)c->alloc((size_t)4 * c->n_tri * sizeof(double));
    }
  }
  if (c->scratch_bytes && !c->scratch) c->scratch = (char*)c->alloc(c->scratch_bytes);
  size_t need = (size_t)slots * c->K * c->iter_tape_bytes;
  if (need > c->tape_cap) {
    c->release(c->tape);
    c->tape_cap = 0;
    c->tape = c->alloc(need);
    c->tape_cap = need;
  }
}

// can `bytes` more of record be held (beyond what the record buffer holds now)?
bool fits_on_device(xpbd_ctx c, size_t bytes) {
  size_t have = c->tape_cap;
  if (bytes <= have) return true;
  size_t extra = bytes - have;
  // adjoint working set not yet allocated counts too (rough upper bound)
  size_t work = c->XB ? 0 : (size_t)c->V * 8 * c->tsz + (size_t)(c->n_dist + c->n_bend + 2 * c->n_tet) * 24 +
                                (size_t)c->n_contact * 6 * c->tsz + (size_t)c->n_tri * (7 * c->tsz + 32);
  if (!c->scratch) work += c->scratch_bytes;
  if (c->budget) return c->dev_bytes + extra + work <= c->budget;
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  const size_t margin = (size_t)8 << 30;   // torch-side tensors of the call (gradients) come on top
  return extra + work + margin <= fr;
}

template <class F> xpbd_status guarded(xpbd_ctx c, F&& fn) {
  try {
    fn();
    if (c) c->err.clear();
    return XPBD_OK;
  } catch (const Fail& f) {
    if (c) c->err = f.msg;
    return f.st;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return XPBD_ERR_OOM;
  } catch (...) {
    if (c) c->err = "unexpected exception";
    return XPBD_ERR_HIP;
  }
}

thread_local std::string g_create_err;

}  // namespace

// ===================================================================== C ABI

extern "C" {

xpbd_status xpbd_create(const xpbd_mesh_desc* mesh, const xpbd_constraint_desc* cons,
                        const xpbd_schedule_desc* schedule, const xpbd_options* opt, xpbd_ctx* out) {
  if (!out) return XPBD_ERR_INVALID;
  *out = nullptr;
  xpbd_ctx c = nullptr;
  try {
    c = new xpbd_ctx_s();
  } catch (...) {
    return XPBD_ERR_OOM;
  }
  xpbd_status st = guarded(c, [&] {
    build(c, mesh, cons, schedule, opt);   // validates everything before it touches the device
    choose_launch(c, opt);
    HIPCHK(hipGetDevice(&c->device));
    if (c->device < 0 || c->device >= kMaxDevices) fail(XPBD_ERR_INVALID, "device %d out of range", c->device);
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      if (!g_scratch_addr[c->device]) {
        void* a = nullptr;
        HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        g_scratch_addr[c->device] = (double*)a;
      }
    }
  });
  if (st != XPBD_OK) {
    g_create_err = c->err;
    delete c;
    return st;
  }
  *out = c;
  return XPBD_OK;
}

xpbd_status xpbd_destroy(xpbd_ctx ctx) {
  if (!ctx) return XPBD_ERR_INVALID;
  if (ctx->in_pack) {
    ctx->err = "destroy: the context is serving a job of a pack";
    return XPBD_ERR_STATE;
  }
  delete ctx;
  return XPBD_OK;
}

xpbd_status xpbd_forward(xpbd_ctx c, const void* x0, const void* v0, const xpbd_params* p, int32_t n_frames,
                         void* x_frames, void* x_final, void* v_final, int32_t flags, void* stream) {
  if (!c) return XPBD_ERR_INVALID;
  return guarded(c, [&] {
    if (c->in_pack) fail(XPBD_ERR_STATE, "forward: the context is serving a job of a pack");
    if (!p || !x0 || !v0 || n_frames < 1) fail(XPBD_ERR_INVALID, "forward: null argument or n_frames < 1");
    if (c->n_tet && !p->tet_E && !(p->tet_mu && p->tet_lambda))
      fail(XPBD_ERR_INVALID, "forward: tet_E, or tet_mu and tet_lambda, required");
    if (!p->tet_mu != !p->tet_lambda) fail(XPBD_ERR_INVALID, "forward: tet_mu and tet_lambda go together");
    if (c->n_tri && !p->tri_coef) fail(XPBD_ERR_INVALID, "forward: tri_coef required");
    if (c->n_bc && !p->body_x) fail(XPBD_ERR_INVALID, "forward: body_x required");
    if (flags & ~XPBD_FWD_FOR_ADJOINT) fail(XPBD_ERR_INVALID, "forward: unknown flags");
    c->have_forward = false;
    c->fwd_recorded = false;
    // how many final frames keep their record: all (whole rollout) if it
    // fits; with tape_mode 0 or 4 otherwise as many as fit (tape_mode 4: at
    // most record_frames), the rest recomputed by the adjoint
    int kept = 0;
    const size_t frame_tape = (size_t)c->S * c->K * c->iter_tape_bytes;
    const int m = c->tape_mode_opt;
    if ((flags & XPBD_FWD_FOR_ADJOINT) && (m == 0 || m == 3 || m == 4)) {
      int cap = n_frames;
      if (m == 4 && c->record_frames_opt > 0) cap = std::min(cap, c->record_frames_opt);
      if (fits_on_device(c, (size_t)cap * frame_tape)) kept = cap;
      if (m == 3 && kept < n_frames)
        fail(XPBD_ERR_OOM, "forward: the record of the whole rollout (%zu bytes) does not fit",
             (size_t)n_frames * frame_tape);
      if (m != 3)
        for (int r = cap - 1; kept == 0 && r >= 1; --r)
          if (fits_on_device(c, (size_t)r * frame_tape)) kept = r;
      if (kept) ensure_adjoint_buffers(c, kept * c->S);
    } else if (m == 3) {
      fail(XPBD_ERR_INVALID, "forward: tape_mode 3 needs XPBD_FWD_FOR_ADJOINT");
    }
    const int rec_from = n_frames - kept;
    hipStream_t st = (hipStream_t)stream;
    if (c->dtype == XPBD_F32) Ops<float>::forward(c, x0, v0, p, n_frames, x_frames, x_final, v_final, rec_from, st);
    else Ops<double>::forward(c, x0, v0, p, n_frames, x_frames, x_final, v_final, rec_from, st);
    c->have_forward = true;
    c->fwd_recorded = kept > 0;
    c->fwd_rec_from = rec_from;
    c->fwd_frames = n_frames;
    c->fwd_params = *p;
  });
}

xpbd_status xpbd_adjoint(xpbd_ctx c, const xpbd_params* p, const void* dLdx_frames, const uint8_t* frame_mask,
                         const void* dLdv_final, const xpbd_grads* out, void* stream) {
  if (!c) return XPBD_ERR_INVALID;
  return guarded(c, [&] {
    if (c->in_pack) fail(XPBD_ERR_STATE, "adjoint: the context is serving a job of a pack");
    if (!p || !out) fail(XPBD_ERR_INVALID, "adjoint: null argument");
    if (!c->have_forward) fail(XPBD_ERR_STATE, "adjoint: no preceding forward on this context");
    const xpbd_params& q = c->fwd_params;
    if (q.dist_compliance != p->dist_compliance || q.bend_compliance != p->bend_compliance ||
        q.tet_E != p->tet_E || q.f_ext != p->f_ext || std::memcmp(q.sphere, p->sphere, sizeof q.sphere) != 0 ||
        q.tet_mu != p->tet_mu || q.tet_lambda != p->tet_lambda || q.tri_coef != p->tri_coef ||
        q.body_x != p->body_x)
      fail(XPBD_ERR_STATE, "adjoint: parameters differ from the preceding forward");
    const int F = c->fwd_frames;
    const int rec_from = c->fwd_recorded ? c->fwd_rec_from : F;
    // the LDS group reverse accumulates the distance and bending compliance
    // adjoints only for a call that asks for one of those gradients
    c->want_ab = out->dist_compliance != nullptr || out->bend_compliance != nullptr;
    // frames without a kept record: recomputed per frame if a frame's record
    // fits (the kept frames' slots are reused once consumed), else per substep
    int mode = c->tape_mode_opt == 1 || c->tape_mode_opt == 2 ? c->tape_mode_opt : 1;
    if (rec_from > 0 && mode == 1 && rec_from == F) {
      size_t frame_tape = (size_t)c->S * c->K * c->iter_tape_bytes;
      if (c->tape_mode_opt != 1 && !fits_on_device(c, frame_tape)) mode = 2;
    }
    if (rec_from > 0 && rec_from < F) mode = 1;   // the kept slots hold at least one frame
    // record slots: the kept frames', and one frame (mode 1) or one substep
    // (mode 2) for the recomputed frames.  With nothing kept, two frames when
    // they fit, so a frame can be recomputed while the next is reversed;
    // kept frames are never moved (growing the record would drop them), and
    // two or more kept frames give the overlap their slots
    int slots = (F - rec_from) * c->S;
    if (rec_from > 0) {
      int want = 1;
      if (mode == 1 && rec_from == F && !c->persistent && !c->serial_adjoint &&
          fits_on_device(c, 2 * (size_t)c->S * c->K * c->iter_tape_bytes))
        want = 2;
      slots = std::max(slots, mode == 1 ? want * c->S : 1);
    }
    ensure_adjoint_buffers(c, slots);
    c->tape_mode_used = rec_from == 0 ? 3 : rec_from < F ? 4 : mode;
    c->fwd_recorded = false;   // a kept record is consumed by this adjoint
    hipStream_t st = (hipStream_t)stream;
    if (c->dtype == XPBD_F32)
      Ops<float>::adjoint(c, p, dLdx_frames, frame_mask, dLdv_final, out, mode, rec_from, st);
    else
      Ops<double>::adjoint(c, p, dLdx_frames, frame_mask, dLdv_final, out, mode, rec_from, st);
  });
}

xpbd_status xpbd_goal_weighted(xpbd_ctx c, const void* x_frames, const void* targets, const uint8_t* frame_mask,
                               const double* vertex_weight, int32_t n_frames, double* loss, void* dLdx,
                               void* stream) {
  if (!c) return XPBD_ERR_INVALID;
  return guarded(c, [&] {
    if (!x_frames || !targets || n_frames < 1) fail(XPBD_ERR_INVALID, "goal: null argument");
    hipStream_t st = (hipStream_t)stream;
    if (c->dtype == XPBD_F32)
      Ops<float>::goal(c, x_frames, targets, frame_mask, vertex_weight, n_frames, loss, dLdx, st);
    else
      Ops<double>::goal(c, x_frames, targets, frame_mask, vertex_weight, n_frames, loss, dLdx, st);
  });
}

xpbd_status xpbd_goal_l2(xpbd_ctx c, const void* x_frames, const void* targets, const uint8_t* frame_mask,
                         int32_t n_frames, double* loss, void* dLdx, void* stream) {
  return xpbd_goal_weighted(c, x_frames, targets, frame_mask, nullptr, n_frames, loss, dLdx, stream);
}

xpbd_status xpbd_goal_weighted_noalloc(xpbd_ctx c, const void* x_frames, const void* targets,
                                       const uint8_t* frame_mask, const double* vertex_weight, int32_t n_frames,
                                       double* loss, void* dLdx, void* stream) {
  if (!c) return XPBD_ERR_INVALID;
  return guarded(c, [&] {
    if (!x_frames || !targets || n_frames < 1) fail(XPBD_ERR_INVALID, "goal: null argument");
    const size_t need = (size_t)nblocks((size_t)3 * c->V) * (size_t)n_frames;
    if (need > kGoalScratchDoubles)
      fail(XPBD_ERR_INVALID, "goal_noalloc: %zu partial sums (3 V / %d per frame x %d frames) exceed the %zu of "
           "the static scratch", need, kBlock, n_frames, kGoalScratchDoubles);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != c->device) fail(XPBD_ERR_INVALID, "goal_noalloc: current device %d, context on device %d", dev,
                               c->device);
    double* parts = g_scratch_addr[c->device];
    hipStream_t st = (hipStream_t)stream;
    if (c->dtype == XPBD_F32)
      Ops<float>::goal_into(c, x_frames, targets, frame_mask, vertex_weight, n_frames, loss, dLdx, parts, st);
    else
      Ops<double>::goal_into(c, x_frames, targets, frame_mask, vertex_weight, n_frames, loss, dLdx, parts, st);
  });
}

xpbd_status xpbd_get_info(xpbd_ctx c, xpbd_info* info) {
  if (!c || !info) return XPBD_ERR_INVALID;
  info->n_verts = c->V;
  info->n_dist = c->n_dist;
  info->n_bend = c->n_bend;
  info->n_tet = c->n_tet;
  info->n_contact = c->n_contact;
  info->n_sets = (int32_t)c->sets.size();
  info->projections_per_iteration = c->proj_per_iter;
  info->device_bytes = (int64_t)c->dev_bytes;
  info->tape_bytes_per_iteration = (int64_t)c->iter_tape_bytes;
  info->tape_mode = c->tape_mode_used;
  info->persistent = c->persistent ? 1 : 0;
  info->persistent_blocks = c->persistent ? c->prog_grid : 0;
  info->n_groups = (int32_t)c->groups.size();
  int nl = 0;
  for (auto& g : c->groups) nl += g.lds ? 1 : 0;
  info->n_groups_lds = nl;
  info->max_group_lds_bytes = c->max_group_lds;
  info->n_materials = c->n_mat;
  info->n_tri = c->n_tri;
  info->n_body_contacts = c->n_bc;
  info->forward_record_frames = c->have_forward ? c->fwd_frames - c->fwd_rec_from : 0;
  info->adjoint_streams = c->adj_streams_used;
  return XPBD_OK;
}

xpbd_status xpbd_profile_enable(xpbd_ctx c, int32_t on) {
  if (!c || on < 0) return XPBD_ERR_INVALID;
  c->prof_stride = on;
  c->prof_counter = 0;
  return XPBD_OK;
}

xpbd_status xpbd_profile_read(xpbd_ctx c, int64_t launches[14], double ms[14], int64_t items[14]) {
  if (!c) return XPBD_ERR_INVALID;
  return guarded(c, [&] {
    for (auto& e : c->ev_pending) {
      HIPCHK(hipEventSynchronize(e.b));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
      c->prof_launch[e.fam] += 1;
      c->prof_ms[e.fam] += t;
      c->prof_items[e.fam] += e.items;
      c->ev_free.push_back({e.a, e.b});
    }
    c->ev_pending.clear();
    for (int i = 0; i < kProfFamilies; ++i) {
      if (launches) launches[i] = c->prof_launch[i];
      if (ms) ms[i] = c->prof_ms[i];
      if (items) items[i] = c->prof_items[i];
      c->prof_launch[i] = 0;
      c->prof_ms[i] = 0;
      c->prof_items[i] = 0;
    }
  });
}

const char* xpbd_last_error(xpbd_ctx c) { return c ? c->err.c_str() : g_create_err.c_str(); }

const char* xpbd_status_string(xpbd_status s) {
  switch (s) {
    case XPBD_OK: return "ok";
    case XPBD_ERR_INVALID: return "invalid argument";
    case XPBD_ERR_OOM: return "out of memory";
    case XPBD_ERR_HIP: return "HIP error";
    case XPBD_ERR_STATE: return "invalid state";
    case XPBD_ERR_NONFINITE: return "non-finite value";
    case XPBD_ERR_SOLVER: return "solver failure";
  }
  return "unknown";
}

}  // extern "C"

#include "xpbd_pack_host.hpp"
#include "xpbd_implicit_host.hpp"
