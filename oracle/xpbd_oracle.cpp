// FP64 reference implementation of differentiable XPBD (DiffXPBD).
//
// TEST INFRASTRUCTURE ONLY.  This file is the checker for the GPU library:
// only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark may load it.  It shares no code with the GPU path.
//
// It is deliberately plain and slow:
//   * every constraint is written once, as the scalar function C(x) of its
//     definition;  gradients and Hessian-vector products come from exact
//     forward-mode automatic differentiation of that one function
//     (a 16-slot gradient dual, nested inside a one-direction dual);
//   * the forward pass follows the XPBD multiplier and position updates
//     (Sec. 3.1, Eq. xpbd and the position update after it) inside the
//     implicit-Euler step of Eq. xpbdUpdateRule, one Gauss-Seidel sweep
//     over the given ordered independent sets per iteration;
//   * the exact adjoint (reverse mode through every substep, iteration and
//     projection) applies the chain rule to each projection in reverse,
//     using the partial derivatives of Sec. 4.3 (dDx/dx, dDlambda/dx, db/dx,
//     dJ/dx) per projection rather than accumulated; the adjoint states
//     follow the recurrence of the supplemental Sec. A (Eq. adjoint_state)
//     and the gradient rule Eq. gradientRule;
//   * an implicit, converged-limit adjoint (Eq. adjointXPBD: one linear
//     solve per step, here dense LU on tiny meshes) is provided as a
//     cross-check of the exact adjoint when the forward solve has converged.
//
// Readings of points the paper leaves open:
//   * distance: C = |xi - xj| - L with L the rest length;
//   * bending: the signed dihedral angle of hinge (x0, x1), wings x2 in
//     triangle (x0, x1, x2) and x3 in (x1, x0, x3), minus its rest value;
//   * Neo-Hookean (Sec. 5.2): C_D = sqrt(tr F^T F), C_H = det F - gamma with
//     gamma = 1 + mu / lambda (or 1), alpha_D = 1/(mu V), alpha_H = 1/(lambda V),
//     D projected before H, separate multipliers;
//   * contact (Sec. 4.5): C = |x - c| - R - tau against a sphere (c, R),
//     projected only while C < 0;
//   * orthotropic StVK membrane (Sec. 5.1): per triangle the vector
//     constraint C = (E_uu, E_vv, 2 E_uv) of the Green strain
//     E = (F^T F - I)/2, F = Ds Dm^-1 (3x2) with Dm the triangle's edges in
//     the warp/weft (u, v) material frame, compliance matrix
//     alpha = (A K)^-1, K = [[C00, C01, 0], [C01, C11, 0], [0, 0, C22]], A the
//     material-space area; projected as one vector XPBD step (a 3x3 solve
//     for the three multipliers);
//   * body collider (Sec. 4.5, 5.3): a triangle mesh with kinematic vertices
//     x_body (a control).  At the start of each substep, after the
//     prediction, every body-contact vertex is paired with the body triangle
//     closest to it (point-triangle distance in FP64, ties to the lower
//     triangle index), or with none if that distance exceeds the search
//     radius; during the substep it keeps C = n . (x - a) - tau >= 0 against
//     the plane of that triangle (a, b, c), n the unit normal of
//     (b - a) x (c - a), projected only while C < 0;
//   * substeps: each substep is one step of Eq. xpbdUpdateRule with
//     dt = frame dt / S; multipliers reset every substep; external force
//     f_ext[f] is constant over the substeps of frame f;  gravity enters as
//     M g, so free vertices get acceleration g and pinned ones (w = 0) none;
//   * a projection whose denominator is zero, or whose constraint is
//     undefined (zero-length edge, degenerate triangle), is skipped.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------ duals
// G: value + 16 partial derivatives.
constexpr int NG = 16;
struct G {
  double v;
  double d[NG];
};
inline G gc(double v) { G r; r.v = v; for (int i = 0; i < NG; ++i) r.d[i] = 0.0; return r; }
inline G gvar(double v, int slot) { G r = gc(v); r.d[slot] = 1.0; return r; }
inline G operator+(const G& a, const G& b) { G r; r.v = a.v + b.v; for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline G operator-(const G& a, const G& b) { G r; r.v = a.v - b.v; for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline G operator-(const G& a) { G r; r.v = -a.v; for (int i = 0; i < NG; ++i) r.d[i] = -a.d[i]; return r; }
inline G operator*(const G& a, const G& b) { G r; r.v = a.v * b.v; for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline G operator/(const G& a, const G& b) { G r; r.v = a.v / b.v; for (int i = 0; i < NG; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
inline G operator*(double s, const G& a) { G r; r.v = s * a.v; for (int i = 0; i < NG; ++i) r.d[i] = s * a.d[i]; return r; }
inline G operator+(const G& a, double s) { G r = a; r.v += s; return r; }
inline G operator-(const G& a, double s) { G r = a; r.v -= s; return r; }
inline G sqrt(const G& a) { G r; r.v = std::sqrt(a.v); for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] / (2.0 * r.v); return r; }
inline G atan2(const G& y, const G& x) {
  G r; r.v = std::atan2(y.v, x.v);
  double den = x.v * x.v + y.v * y.v;
  for (int i = 0; i < NG; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
  return r;
}
inline double val(double a) { return a; }
inline double val(const G& a) { return a.v; }

// H: one-direction dual over G (value part and directional-derivative part).
struct H { G v, t; };
inline H hc(double v) { return H{gc(v), gc(0.0)}; }
inline H operator+(const H& a, const H& b) { return H{a.v + b.v, a.t + b.t}; }
inline H operator-(const H& a, const H& b) { return H{a.v - b.v, a.t - b.t}; }
inline H operator-(const H& a) { return H{-a.v, -a.t}; }
inline H operator*(const H& a, const H& b) { return H{a.v * b.v, a.t * b.v + a.v * b.t}; }
inline H operator/(const H& a, const H& b) { return H{a.v / b.v, (a.t * b.v - a.v * b.t) / (b.v * b.v)}; }
inline H operator*(double s, const H& a) { return H{s * a.v, s * a.t}; }
inline H operator+(const H& a, double s) { return H{a.v + s, a.t}; }
inline H operator-(const H& a, double s) { return H{a.v - s, a.t}; }
inline H sqrt(const H& a) { G s = sqrt(a.v); return H{s, a.t / (2.0 * s)}; }
inline H atan2(const H& y, const H& x) {
  G r = atan2(y.v, x.v);
  G den = x.v * x.v + y.v * y.v;
  return H{r, (x.v * y.t - y.v * x.t) / den};
}
inline double val(const H& a) { return a.v.v; }
using std::sqrt;
using std::atan2;

template <class S> struct V3 { S x, y, z; };
template <class S> V3<S> sub(const V3<S>& a, const V3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ------------------------------------------------------------------ constraints
// Each returns C and reports whether C is defined at this configuration.

template <class S> S c_distance(const V3<S>* p, double L, bool* ok) {
  V3<S> r = sub(p[0], p[1]);
  S len2 = dot(r, r);
  *ok = val(len2) > 0.0;
  if (!*ok) return len2;
  return sqrt(len2) - L;
}

// signed dihedral angle: n1 = (x1-x0) x (x2-x0), n2 = (x0-x1) x (x3-x1),
// theta = atan2(((n1 x n2) . e) / |e|, n1 . n2) with e = x1 - x0.
template <class S> S dihedral(const V3<S>* p, bool* ok) {
  V3<S> e = sub(p[1], p[0]);
  V3<S> n1 = cross(e, sub(p[2], p[0]));
  V3<S> n2 = cross(sub(p[0], p[1]), sub(p[3], p[1]));
  S le2 = dot(e, e);
  *ok = val(le2) > 0.0 && val(dot(n1, n1)) > 0.0 && val(dot(n2, n2)) > 0.0;
  if (!*ok) return le2;
  S y = dot(cross(n1, n2), e) / sqrt(le2);
  S x = dot(n1, n2);
  return atan2(y, x);
}
template <class S> S c_bend(const V3<S>* p, double theta0, bool* ok) {
  S th = dihedral(p, ok);
  return th - theta0;
}

// F = Ds B, Ds = [x1-x0, x2-x0, x3-x0] (columns), B = Dm^-1 (row-major 3x3).
template <class S> void deformation_gradient(const V3<S>* p, const double* B, S F[3][3]) {
  V3<S> c[3] = {sub(p[1], p[0]), sub(p[2], p[0]), sub(p[3], p[0])};
  for (int r = 0; r < 3; ++r) {
    for (int col = 0; col < 3; ++col) {
      S acc = (r == 0 ? c[0].x : r == 1 ? c[0].y : c[0].z) * B[0 * 3 + col];
      acc = acc + (r == 0 ? c[1].x : r == 1 ? c[1].y : c[1].z) * B[1 * 3 + col];
      acc = acc + (r == 0 ? c[2].x : r == 1 ? c[2].y : c[2].z) * B[2 * 3 + col];
      F[r][col] = acc;
    }
  }
}
inline G operator*(const G& a, double s) { return s * a; }
inline H operator*(const H& a, double s) { return s * a; }

template <class S> S c_tet_dev(const V3<S>* p, const double* B, bool* ok) {
  S F[3][3];
  deformation_gradient(p, B, F);
  S acc = F[0][0] * F[0][0];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      if (r || c) acc = acc + F[r][c] * F[r][c];
  *ok = val(acc) > 0.0;
  if (!*ok) return acc;
  return sqrt(acc);
}
template <class S> S c_tet_hyd(const V3<S>* p, const double* B, double gamma, bool* ok) {
  S F[3][3];
  deformation_gradient(p, B, F);
  S det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1])
        - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0])
        + F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  *ok = true;
  return det - gamma;
}
// sphere: variables are x (3) then c (3) then R (1)
template <class S> S c_contact(const V3<S>& x, const V3<S>& c, const S& R, double tau, bool* ok) {
  V3<S> r = sub(x, c);
  S d2 = dot(r, r);
  *ok = val(d2) > 0.0;
  if (!*ok) return d2;
  return sqrt(d2) - R - tau;
}

// Green strain of a membrane triangle in Voigt form, component comp:
// 0 -> E_uu, 1 -> E_vv, 2 -> 2 E_uv, with E = (F^T F - I)/2 and
// F = [x1-x0, x2-x0] Bm (3x2), Bm = Dm^-1 row-major 2x2.
template <class S> S c_membrane(const V3<S>* p, const double* Bm, int comp, bool* ok) {
  *ok = true;
  V3<S> d1 = sub(p[1], p[0]), d2 = sub(p[2], p[0]);
  V3<S> fu = {d1.x * Bm[0] + d2.x * Bm[2], d1.y * Bm[0] + d2.y * Bm[2], d1.z * Bm[0] + d2.z * Bm[2]};
  V3<S> fv = {d1.x * Bm[1] + d2.x * Bm[3], d1.y * Bm[1] + d2.y * Bm[3], d1.z * Bm[1] + d2.z * Bm[3]};
  if (comp == 0) return 0.5 * (dot(fu, fu) - 1.0);
  if (comp == 1) return 0.5 * (dot(fv, fv) - 1.0);
  return dot(fu, fv);
}

// Body contact: signed distance of x to the plane of triangle (a, b, c)
// minus the thickness; undefined for a degenerate triangle.
template <class S> S c_body(const V3<S>& x, const V3<S>& a, const V3<S>& b, const V3<S>& c, double tau, bool* ok) {
  V3<S> n = cross(sub(b, a), sub(c, a));
  S n2 = dot(n, n);
  *ok = val(n2) > 0.0;
  if (!*ok) return n2;
  return dot(n, sub(x, a)) / sqrt(n2) - tau;
}

// Squared distance from p to the segment [a, b]: to the orthogonal
// projection of p onto the segment's line, clamped to the segment.
double point_segment_d2(const V3<double>& p, const V3<double>& a, const V3<double>& b) {
  V3<double> ab = sub(b, a);
  double L2 = dot(ab, ab);
  double t = L2 > 0.0 ? dot(sub(p, a), ab) / L2 : 0.0;
  t = std::min(1.0, std::max(0.0, t));
  V3<double> r = sub(p, {a.x + t * ab.x, a.y + t * ab.y, a.z + t * ab.z});
  return dot(r, r);
}

// Squared distance from p to triangle (a, b, c), from the definition of the
// distance to a set: when the orthogonal projection q of p onto the
// triangle's plane lies in the triangle (the signed areas of q with each edge
// all have the sign of the triangle's) the distance is |p - q|; otherwise the
// closest point is on the boundary, and the distance is the least of the
// distances to the three edges.
double point_triangle_d2(const V3<double>& p, const V3<double>& a, const V3<double>& b, const V3<double>& c) {
  V3<double> n = cross(sub(b, a), sub(c, a));
  double nn = dot(n, n);
  if (nn > 0.0) {
    double s = dot(sub(p, a), n) / nn;
    V3<double> q = {p.x - s * n.x, p.y - s * n.y, p.z - s * n.z};
    double wa = dot(cross(sub(b, q), sub(c, q)), n);
    double wb = dot(cross(sub(c, q), sub(a, q)), n);
    double wc = dot(cross(sub(a, q), sub(b, q)), n);
    if (wa >= 0.0 && wb >= 0.0 && wc >= 0.0) {
      V3<double> r = sub(p, q);
      return dot(r, r);
    }
  }
  return std::min(point_segment_d2(p, a, b), std::min(point_segment_d2(p, b, c), point_segment_d2(p, c, a)));
}

// ------------------------------------------------------------------ scene ABI
struct Scene {
  int32_t n_verts;
  const double* rest;
  const double* inv_mass;
  int32_t n_dist; const int32_t* dist_v;
  int32_t n_bend; const int32_t* bend_v;
  int32_t n_tet; const int32_t* tet_v; const double* tet_nu;
  int32_t contact; double contact_thickness; double contact_compliance;
  int32_t n_sets; const int32_t* set_type; const int64_t* set_off; const int32_t* set_items;
  double dt; int32_t substeps; int32_t iterations; double gravity[3];
  int32_t tet_gamma_one;
  int32_t emulate_f32;
  int32_t n_threads;
  int32_t n_tri; const int32_t* tri_v; const double* tri_uv;   // membrane triangles, uv [n_tri][3][2]
  int32_t n_body_verts; int32_t n_body_tris; const int32_t* body_tris;   // body collider mesh
  double body_thickness; double body_compliance; double body_radius;
};
struct Params {
  const double* dist_alpha;
  const double* bend_alpha;
  const double* tet_E;
  const double* f_ext;   // [F][V][3] or null
  double sphere[4];
  // Lame parameters per tet (Sec. 5.2); when given they replace (E, nu)
  const double* tet_mu;
  const double* tet_lambda;
  const double* tri_coef;   // [n_tri][4] = C00, C01, C11, C22
  const double* body_x;     // [n_body_verts][3] body vertex positions
};

enum { T_DIST = 0, T_BEND = 1, T_TET = 2, T_CONTACT = 3, T_TRI = 4, T_BODY = 5 };

// one scalar constraint row ("projection"): a tet item holds two (D then H)
struct Row {
  int type;       // T_DIST, T_BEND, T_TET (sub = 0 dev, 1 hyd), T_CONTACT
  int sub;
  int item;       // constraint index within its type
  int nv;         // vertices touched
  int v[4];
  int lam;        // multiplier slot
};

struct Model {
  const Scene* s;
  std::vector<double> L;       // rest lengths
  std::vector<double> theta0;  // rest dihedral angles
  std::vector<double> B;       // [n_tet][9]
  std::vector<double> vol;     // [n_tet]
  std::vector<double> mu, lam; // per tet, from E (filled per call)
  std::vector<double> gamma;
  std::vector<double> tB;      // [n_tri][4] Dm^-1 of each membrane triangle (row-major 2x2)
  std::vector<double> tarea;   // [n_tri] material-space area
  int lam_tri = 0;             // membrane multipliers: 3 per triangle
  int lam_body = 0;            // body-contact multipliers, one per listed vertex
  std::vector<int> body_slot;  // vertex -> body-contact multiplier slot (-1: none)
  int n_lam;
  int lam_dist, lam_bend, lam_tet, lam_contact;  // offsets of each type's multipliers
  std::vector<int> contact_slot;                 // vertex -> contact multiplier slot
};

inline double rnd(const Scene* s, double x) { return s->emulate_f32 ? (double)(float)x : x; }

V3<double> vtx(const double* x, int k) { return {x[3 * k], x[3 * k + 1], x[3 * k + 2]}; }

int build_model(const Scene* s, Model* m) {
  m->s = s;
  const int V = s->n_verts;
  m->L.resize(s->n_dist);
  for (int e = 0; e < s->n_dist; ++e) {
    int i = s->dist_v[2 * e], j = s->dist_v[2 * e + 1];
    if (i < 0 || j < 0 || i >= V || j >= V) return 1;
    V3<double> r = sub(vtx(s->rest, i), vtx(s->rest, j));
    m->L[e] = std::sqrt(dot(r, r));
  }
  m->theta0.resize(s->n_bend);
  for (int b = 0; b < s->n_bend; ++b) {
    V3<double> p[4];
    for (int k = 0; k < 4; ++k) {
      int vi = s->bend_v[4 * b + k];
      if (vi < 0 || vi >= V) return 1;
      p[k] = vtx(s->rest, vi);
    }
    bool ok;
    double th = dihedral(p, &ok);
    if (!ok) return 1;
    m->theta0[b] = th;
  }
  m->B.resize(9 * (size_t)s->n_tet);
  m->vol.resize(s->n_tet);
  for (int t = 0; t < s->n_tet; ++t) {
    V3<double> p[4];
    for (int k = 0; k < 4; ++k) {
      int vi = s->tet_v[4 * t + k];
      if (vi < 0 || vi >= V) return 1;
      p[k] = vtx(s->rest, vi);
    }
    // Dm columns = rest edge vectors
    double D[3][3];
    V3<double> c[3] = {sub(p[1], p[0]), sub(p[2], p[0]), sub(p[3], p[0])};
    for (int col = 0; col < 3; ++col) { D[0][col] = c[col].x; D[1][col] = c[col].y; D[2][col] = c[col].z; }
    double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1])
               - D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0])
               + D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    if (!(det > 0.0)) return 1;
    // inverse by the adjugate
    double* Bt = &m->B[9 * (size_t)t];
    Bt[0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) / det;
    Bt[1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) / det;
    Bt[2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) / det;
    Bt[3] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) / det;
    Bt[4] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) / det;
    Bt[5] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) / det;
    Bt[6] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) / det;
    Bt[7] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) / det;
    Bt[8] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) / det;
    m->vol[t] = det / 6.0;
  }
  m->lam_dist = 0;
  m->lam_bend = s->n_dist;
  m->lam_tet = s->n_dist + s->n_bend;
  m->lam_contact = m->lam_tet + 2 * s->n_tet;
  m->contact_slot.assign(V, -1);
  int nc = 0;
  if (s->contact)
    for (int k = 0; k < V; ++k)
      if (s->inv_mass[k] > 0.0) m->contact_slot[k] = nc++;
  m->n_lam = m->lam_contact + nc;
  m->tB.resize(4 * (size_t)s->n_tri);
  m->tarea.resize(s->n_tri);
  for (int t = 0; t < s->n_tri; ++t) {
    for (int k = 0; k < 3; ++k)
      if (s->tri_v[3 * t + k] < 0 || s->tri_v[3 * t + k] >= V) return 1;
    const double* uv = s->tri_uv + 6 * (size_t)t;
    // Dm columns = material-space edges (u1-u0, v1-v0) and (u2-u0, v2-v0)
    double a = uv[2] - uv[0], b = uv[4] - uv[0], cc = uv[3] - uv[1], d = uv[5] - uv[1];
    double det = a * d - b * cc;
    if (!(std::fabs(det) > 0.0)) return 1;
    double* Bt = &m->tB[4 * (size_t)t];
    Bt[0] = d / det; Bt[1] = -b / det; Bt[2] = -cc / det; Bt[3] = a / det;
    m->tarea[t] = 0.5 * std::fabs(det);
  }
  m->lam_tri = m->n_lam;
  m->n_lam += 3 * s->n_tri;
  for (int64_t i = 0; i < 3 * (int64_t)s->n_body_tris; ++i)
    if (s->body_tris[i] < 0 || s->body_tris[i] >= s->n_body_verts) return 1;
  m->lam_body = m->n_lam;
  m->body_slot.assign(V, -1);
  for (int si = 0; si < s->n_sets; ++si)
    if (s->set_type[si] == T_BODY)
      for (int64_t q = s->set_off[si]; q < s->set_off[si + 1]; ++q) {
        int it = s->set_items[q];
        if (it < 0 || it >= V || s->inv_mass[it] <= 0.0 || m->body_slot[it] >= 0) return 1;
        m->body_slot[it] = m->n_lam++;
      }
  // schedule check: every set's type valid and items in range
  for (int si = 0; si < s->n_sets; ++si) {
    int ty = s->set_type[si];
    if (ty < T_DIST || ty > T_BODY) return 1;
    if (ty == T_BODY) continue;   // checked above
    int lim = ty == T_DIST ? s->n_dist : ty == T_BEND ? s->n_bend : ty == T_TET ? s->n_tet : ty == T_TRI ? s->n_tri : V;
    for (int64_t q = s->set_off[si]; q < s->set_off[si + 1]; ++q) {
      int it = s->set_items[q];
      if (it < 0 || it >= lim) return 1;
      if (ty == T_CONTACT && m->contact_slot[it] < 0) return 1;
    }
  }
  return 0;
}

void set_materials(Model* m, const Params* p) {
  const Scene* s = m->s;
  m->mu.resize(s->n_tet); m->lam.resize(s->n_tet); m->gamma.resize(s->n_tet);
  for (int t = 0; t < s->n_tet; ++t) {
    if (p->tet_mu) {
      m->mu[t] = p->tet_mu[t];
      m->lam[t] = p->tet_lambda[t];
    } else {
      double E = p->tet_E[t], nu = s->tet_nu[t];
      m->mu[t] = E / (2.0 * (1.0 + nu));
      m->lam[t] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    }
    m->gamma[t] = s->tet_gamma_one ? 1.0 : 1.0 + m->mu[t] / m->lam[t];
  }
}

Row make_row(const Model& mm, int type, int item, int sub) {
  const Model* m = &mm;
  const Scene* s = m->s;
  Row r{}; r.type = type; r.item = item; r.sub = sub;
  if (type == T_DIST) { r.nv = 2; r.v[0] = s->dist_v[2 * item]; r.v[1] = s->dist_v[2 * item + 1]; r.lam = m->lam_dist + item; }
  else if (type == T_BEND) { r.nv = 4; for (int k = 0; k < 4; ++k) r.v[k] = s->bend_v[4 * item + k]; r.lam = m->lam_bend + item; }
  else if (type == T_TET) { r.nv = 4; for (int k = 0; k < 4; ++k) r.v[k] = s->tet_v[4 * item + k]; r.lam = m->lam_tet + 2 * item + sub; }
  else if (type == T_TRI) { r.nv = 3; for (int k = 0; k < 3; ++k) r.v[k] = s->tri_v[3 * item + k]; r.lam = m->lam_tri + 3 * item; }
  else if (type == T_BODY) { r.nv = 1; r.v[0] = item; r.lam = m->body_slot[item]; }
  else { r.nv = 1; r.v[0] = item; r.lam = m->lam_contact + m->contact_slot[item]; }
  return r;
}

double row_compliance(const Model* m, const Params* p, const Row& r) {
  const Scene* s = m->s;
  if (r.type == T_DIST) return rnd(s, p->dist_alpha[r.item]);
  if (r.type == T_BEND) return rnd(s, p->bend_alpha[r.item]);
  if (r.type == T_TET) {
    double a = r.sub == 0 ? 1.0 / (m->mu[r.item] * m->vol[r.item]) : 1.0 / (m->lam[r.item] * m->vol[r.item]);
    return rnd(s, a);
  }
  return s->contact_compliance;
}

// Evaluate C of a row with scalar type S; variables: positions of the row's
// vertices (slots 3k..3k+2), then for contact the sphere centre (12..14) and
// radius (15).
template <class S> S eval_row(const Model* m, const Row& r, const V3<S>* p, const V3<S>& cs, const S& R, bool* ok) {
  const Scene* s = m->s;
  if (r.type == T_DIST) return c_distance(p, m->L[r.item], ok);
  if (r.type == T_BEND) return c_bend(p, m->theta0[r.item], ok);
  if (r.type == T_TET) {
    const double* B = &m->B[9 * (size_t)r.item];
    return r.sub == 0 ? c_tet_dev(p, B, ok) : c_tet_hyd(p, B, m->gamma[r.item], ok);
  }
  if (r.type == T_TRI) return c_membrane(p, &m->tB[4 * (size_t)r.item], r.sub, ok);
  return c_contact(p[0], cs, R, s->contact_thickness, ok);
}

// C and all 16 partials at x.
struct Eval { bool ok; double C; double g[NG]; };
Eval eval_grad(const Model* m, const Params* P, const Row& r, const double* x) {
  V3<G> p[4];
  for (int k = 0; k < r.nv; ++k)
    p[k] = {gvar(x[3 * r.v[k]], 3 * k), gvar(x[3 * r.v[k] + 1], 3 * k + 1), gvar(x[3 * r.v[k] + 2], 3 * k + 2)};
  V3<G> cs = {gvar(P->sphere[0], 12), gvar(P->sphere[1], 13), gvar(P->sphere[2], 14)};
  G R = gvar(P->sphere[3], 15);
  Eval e;
  G c = eval_row(m, r, p, cs, R, &e.ok);
  e.C = c.v;
  for (int i = 0; i < NG; ++i) e.g[i] = c.d[i];
  return e;
}
// Hessian of C times the direction gdir (16 slots) at x, via the nested dual.
void eval_hvp(const Model* m, const Params* P, const Row& r, const double* x, const double* gdir, double* hv) {
  V3<H> p[4];
  for (int k = 0; k < r.nv; ++k) {
    H c3[3];
    for (int a = 0; a < 3; ++a) c3[a] = H{gvar(x[3 * r.v[k] + a], 3 * k + a), gc(gdir[3 * k + a])};
    p[k] = {c3[0], c3[1], c3[2]};
  }
  V3<H> cs = {H{gvar(P->sphere[0], 12), gc(gdir[12])}, H{gvar(P->sphere[1], 13), gc(gdir[13])},
              H{gvar(P->sphere[2], 14), gc(gdir[14])}};
  H R{gvar(P->sphere[3], 15), gc(gdir[15])};
  bool ok;
  H c = eval_row(m, r, p, cs, R, &ok);
  for (int i = 0; i < NG; ++i) hv[i] = c.t.d[i];
}

// ------------------------------------------------------------------ forward

// a tape entry: the positions of the row's vertices and its multiplier
// before the projection, plus whether it was applied
struct TapeEntry { double x[12]; double lam; double lamv[3]; int tri; };

struct Ctx {
  Model m;
  const Params* p;
  double h;
  std::vector<int>* pair = nullptr;   // vertex -> paired body triangle of this substep (-1: none)
};

// ---- body collider
V3<double> body_vtx(const Ctx& c, int k) { const double* b = c.p->body_x; return {b[3 * k], b[3 * k + 1], b[3 * k + 2]}; }

// pair every body-contact vertex with its closest body triangle (brute force)
void body_detect(const Ctx& c, const double* x) {
  const Scene* s = c.m.s;
  std::vector<int>& pr = *c.pair;
  pr.assign(s->n_verts, -1);
  const double r2 = s->body_radius * s->body_radius;
#pragma omp parallel for schedule(static) num_threads(s->n_threads > 0 ? s->n_threads : 1)
  for (int k = 0; k < s->n_verts; ++k) {
    if (c.m.body_slot[k] < 0) continue;
    V3<double> p = {x[3 * k], x[3 * k + 1], x[3 * k + 2]};
    // the least distance, then the lowest-index triangle within a rounding
    // margin of it (a point nearest to an edge or corner shared by several
    // triangles is equally near to each of them)
    std::vector<double> d2(s->n_body_tris);
    double bd = INFINITY;
    for (int t = 0; t < s->n_body_tris; ++t) {
      const int32_t* q = s->body_tris + 3 * (int64_t)t;
      d2[t] = point_triangle_d2(p, body_vtx(c, q[0]), body_vtx(c, q[1]), body_vtx(c, q[2]));
      bd = std::min(bd, d2[t]);
    }
    int best = -1;
    if (bd <= r2)
      for (int t = 0; t < s->n_body_tris && best < 0; ++t)
        if (d2[t] <= bd * (1.0 + 1e-9) + 1e-20) best = t;
    pr[k] = best;
  }
}

struct BodyEval { bool ok; double C; double g[NG]; };
// C and its partials: slots 0..2 the cloth vertex, 3..11 the triangle's corners
BodyEval body_eval(const Ctx& c, const double* xk, int tri) {
  const int32_t* q = c.m.s->body_tris + 3 * (int64_t)tri;
  V3<G> v[4];
  v[0] = {gvar(xk[0], 0), gvar(xk[1], 1), gvar(xk[2], 2)};
  for (int j = 0; j < 3; ++j) {
    V3<double> b = body_vtx(c, q[j]);
    v[1 + j] = {gvar(b.x, 3 + 3 * j), gvar(b.y, 4 + 3 * j), gvar(b.z, 5 + 3 * j)};
  }
  BodyEval e;
  G cc = c_body(v[0], v[1], v[2], v[3], c.m.s->body_thickness, &e.ok);
  e.C = cc.v;
  for (int i = 0; i < NG; ++i) e.g[i] = cc.d[i];
  return e;
}
void body_hvp(const Ctx& c, const double* xk, int tri, const double* gdir, double* hv) {
  const int32_t* q = c.m.s->body_tris + 3 * (int64_t)tri;
  V3<H> v[4];
  H c0[3];
  for (int a = 0; a < 3; ++a) c0[a] = H{gvar(xk[a], a), gc(gdir[a])};
  v[0] = {c0[0], c0[1], c0[2]};
  for (int j = 0; j < 3; ++j) {
    V3<double> b = body_vtx(c, q[j]);
    double bb[3] = {b.x, b.y, b.z};
    H cj[3];
    for (int a = 0; a < 3; ++a) cj[a] = H{gvar(bb[a], 3 + 3 * j + a), gc(gdir[3 + 3 * j + a])};
    v[1 + j] = {cj[0], cj[1], cj[2]};
  }
  bool ok;
  H cc = c_body(v[0], v[1], v[2], v[3], c.m.s->body_thickness, &ok);
  for (int i = 0; i < NG; ++i) hv[i] = cc.t.d[i];
}
void project_body(const Ctx& c, int k, double* x, double* lam, TapeEntry* tape) {
  const Scene* s = c.m.s;
  const int slot = c.m.body_slot[k];
  const int tri = (*c.pair)[k];
  if (tape) {
    for (int a = 0; a < 3; ++a) tape->x[a] = x[3 * k + a];
    tape->lam = lam[slot];
    tape->tri = tri;
  }
  if (tri < 0) return;
  BodyEval e = body_eval(c, x + 3 * k, tri);
  if (!e.ok || e.C >= 0.0) return;
  const double w = s->inv_mass[k];
  const double at = s->body_compliance / (c.h * c.h);
  const double D = w * (e.g[0] * e.g[0] + e.g[1] * e.g[1] + e.g[2] * e.g[2]) + at;
  if (D == 0.0) return;
  const double dl = (-e.C - at * lam[slot]) / D;
  lam[slot] = rnd(s, lam[slot] + dl);
  for (int a = 0; a < 3; ++a) x[3 * k + a] = rnd(s, x[3 * k + a] + w * dl * e.g[a]);
}
// reverse of one body-contact projection; the body corners' adjoints go to
// part[9] (corner j, axis a at 3 j + a)
void reverse_body(const Ctx& c, int k, const TapeEntry& te, double* xb, double* lamb, double* part) {
  const Scene* s = c.m.s;
  const int slot = c.m.body_slot[k];
  if (te.tri < 0) return;
  BodyEval e = body_eval(c, te.x, te.tri);
  if (!e.ok || e.C >= 0.0) return;
  const double w = s->inv_mass[k];
  const double at = s->body_compliance / (c.h * c.h);
  const double D = w * (e.g[0] * e.g[0] + e.g[1] * e.g[1] + e.g[2] * e.g[2]) + at;
  if (D == 0.0) return;
  const double lb = te.lam;
  const double dl = (-e.C - at * lb) / D;
  double dlb = lamb[slot];
  for (int a = 0; a < 3; ++a) dlb += w * e.g[a] * xb[3 * k + a];
  double gbar[NG] = {0};   // adjoint of grad_x C (the corners do not move)
  for (int a = 0; a < 3; ++a) gbar[a] = w * dl * xb[3 * k + a] - 2.0 * w * e.g[a] * dlb * dl / D;
  const double Cbar = -dlb / D;
  lamb[slot] = lamb[slot] - dlb * at / D;
  double hv[NG];
  body_hvp(c, te.x, te.tri, gbar, hv);
  for (int a = 0; a < 3; ++a) xb[3 * k + a] += Cbar * e.g[a] + hv[a];
  for (int i = 0; i < 9; ++i) part[i] += Cbar * e.g[3 + i] + hv[3 + i];
}

// ---- membrane triangles: one vector projection
// 3x3 helpers (row-major)
void solve3(const double A[9], const double b[3], double xo[3]) {
  // Gaussian elimination with partial pivoting
  double M[3][4];
  for (int i = 0; i < 3; ++i) { for (int j = 0; j < 3; ++j) M[i][j] = A[3 * i + j]; M[i][3] = b[i]; }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int i = col + 1; i < 3; ++i) if (std::fabs(M[i][col]) > std::fabs(M[piv][col])) piv = i;
    if (piv != col) for (int j = 0; j < 4; ++j) std::swap(M[col][j], M[piv][j]);
    for (int i = col + 1; i < 3; ++i) {
      double f = M[i][col] / M[col][col];
      for (int j = col; j < 4; ++j) M[i][j] -= f * M[col][j];
    }
  }
  for (int i = 2; i >= 0; --i) {
    double acc = M[i][3];
    for (int j = i + 1; j < 3; ++j) acc -= M[i][j] * xo[j];
    xo[i] = acc / M[i][i];
  }
}
void inverse3(const double A[9], double Ai[9]) {
  for (int j = 0; j < 3; ++j) {
    double e[3] = {0, 0, 0}, col[3];
    e[j] = 1.0;
    solve3(A, e, col);
    for (int i = 0; i < 3; ++i) Ai[3 * i + j] = col[i];
  }
}
// compliance matrix alpha = (A K)^-1 of triangle t
void membrane_alpha(const Ctx& c, int t, double al[9]) {
  const double* q = c.p->tri_coef + 4 * (size_t)t;
  double A = c.m.tarea[t];
  double K[9] = {A * q[0], A * q[1], 0.0, A * q[1], A * q[2], 0.0, 0.0, 0.0, A * q[3]};
  inverse3(K, al);
  for (int i = 0; i < 9; ++i) al[i] = rnd(c.m.s, al[i]);
}
struct MemEval { double C[3]; double G[3][9]; double J[9]; double at[9]; double w[3]; };
// C, its 3x9 Jacobian, at = alpha / h^2 and J = G W G^T + at at positions xl
void membrane_eval(const Ctx& c, const Row& r, const double* xl, MemEval& e) {
  const Scene* s = c.m.s;
  Row rl = r;
  for (int k = 0; k < 3; ++k) rl.v[k] = k;
  for (int comp = 0; comp < 3; ++comp) {
    rl.sub = comp;
    Eval ev = eval_grad(&c.m, c.p, rl, xl);
    e.C[comp] = ev.C;
    for (int i = 0; i < 9; ++i) e.G[comp][i] = ev.g[i];
  }
  double al[9];
  membrane_alpha(c, r.item, al);
  for (int i = 0; i < 9; ++i) e.at[i] = al[i] / (c.h * c.h);
  for (int k = 0; k < 3; ++k) e.w[k] = s->inv_mass[r.v[k]];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = e.at[3 * a + b];
      for (int i = 0; i < 9; ++i) acc += e.G[a][i] * e.w[i / 3] * e.G[b][i];
      e.J[3 * a + b] = acc;
    }
}
void project_membrane(const Ctx& c, const Row& r, double* x, double* lam, TapeEntry* tape) {
  const Scene* s = c.m.s;
  double xl[9];
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 3; ++a) xl[3 * k + a] = x[3 * r.v[k] + a];
  if (tape) {
    for (int i = 0; i < 9; ++i) tape->x[i] = xl[i];
    for (int a = 0; a < 3; ++a) tape->lamv[a] = lam[r.lam + a];
  }
  MemEval e;
  membrane_eval(c, r, xl, e);
  double b[3], dl[3];
  for (int a = 0; a < 3; ++a) {
    b[a] = -e.C[a];
    for (int q = 0; q < 3; ++q) b[a] -= e.at[3 * a + q] * lam[r.lam + q];
  }
  solve3(e.J, b, dl);
  for (int a = 0; a < 3; ++a) lam[r.lam + a] = rnd(s, lam[r.lam + a] + dl[a]);
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 3; ++a) {
      double dx = 0.0;
      for (int q = 0; q < 3; ++q) dx += e.G[q][3 * k + a] * dl[q];
      double& xv = x[3 * r.v[k] + a];
      xv = rnd(s, xv + e.w[k] * dx);
    }
}

// project one row in place (x, lam); returns true if applied.
bool project_row(const Ctx& c, const Row& r, double* x, double* lam, TapeEntry* tape) {
  const Scene* s = c.m.s;
  if (r.type == T_TRI) { project_membrane(c, r, x, lam, tape); return true; }
  if (r.type == T_BODY) { project_body(c, r.item, x, lam, tape); return true; }
  if (tape) {
    for (int k = 0; k < r.nv; ++k)
      for (int a = 0; a < 3; ++a) tape->x[3 * k + a] = x[3 * r.v[k] + a];
    tape->lam = lam[r.lam];
  }
  Eval e = eval_grad(&c.m, c.p, r, x);
  if (!e.ok) return false;
  if (r.type == T_CONTACT && e.C >= 0.0) return false;
  double at = row_compliance(&c.m, c.p, r) / (c.h * c.h);
  double D = at;
  for (int k = 0; k < r.nv; ++k) {
    double w = s->inv_mass[r.v[k]];
    D += w * (e.g[3 * k] * e.g[3 * k] + e.g[3 * k + 1] * e.g[3 * k + 1] + e.g[3 * k + 2] * e.g[3 * k + 2]);
  }
  if (D == 0.0) return false;
  double dl = (-e.C - at * lam[r.lam]) / D;
  lam[r.lam] = rnd(s, lam[r.lam] + dl);
  for (int k = 0; k < r.nv; ++k) {
    double w = s->inv_mass[r.v[k]];
    for (int a = 0; a < 3; ++a) {
      double& xv = x[3 * r.v[k] + a];
      xv = rnd(s, xv + w * dl * e.g[3 * k + a]);
    }
  }
  return true;
}

int set_rows(const Model& m, int si) { return m.s->set_type[si] == T_TET ? 2 : 1; }

// One Gauss-Seidel sweep (all sets in order).  If tape != null, entries are
// appended in (set, item, sub) order.
void sweep(const Ctx& c, double* x, double* lam, std::vector<TapeEntry>* tape) {
  const Scene* s = c.m.s;
  for (int si = 0; si < s->n_sets; ++si) {
    int ty = s->set_type[si];
    int64_t b = s->set_off[si], e = s->set_off[si + 1];
    int nsub = set_rows(c.m, si);
    size_t base = 0;
    if (tape) { base = tape->size(); tape->resize(base + (size_t)(e - b) * nsub); }
#pragma omp parallel for schedule(static) num_threads(s->n_threads > 0 ? s->n_threads : 1)
    for (int64_t q = b; q < e; ++q) {
      for (int sub = 0; sub < nsub; ++sub) {
        Row r = make_row(c.m, ty, s->set_items[q], sub);
        TapeEntry* te = tape ? &(*tape)[base + (size_t)(q - b) * nsub + sub] : nullptr;
        project_row(c, r, x, lam, te);
      }
    }
  }
}

// One substep of Eq. xpbdUpdateRule.  f: this frame's force [V][3] or null.
void substep(const Ctx& c, double* x, double* v, double* lam, const double* f,
             std::vector<TapeEntry>* tape, std::vector<double>* xprev_out) {
  const Scene* s = c.m.s;
  const int V = s->n_verts;
  const double h = c.h;
  std::vector<double> xprev(x, x + 3 * (size_t)V);
  for (int k = 0; k < V; ++k) {
    double w = s->inv_mass[k];
    if (w > 0.0) {
      for (int a = 0; a < 3; ++a) {
        double fa = f ? f[3 * k + a] : 0.0;
        v[3 * k + a] = rnd(s, v[3 * k + a] + h * (s->gravity[a] + w * fa));
      }
    }
    for (int a = 0; a < 3; ++a) x[3 * k + a] = rnd(s, x[3 * k + a] + h * v[3 * k + a]);
  }
  std::fill(lam, lam + c.m.n_lam, 0.0);
  if (c.pair) body_detect(c, x);
  for (int it = 0; it < s->iterations; ++it) sweep(c, x, lam, tape);
  for (size_t i = 0; i < 3 * (size_t)V; ++i) v[i] = rnd(s, (x[i] - xprev[i]) / h);
  if (xprev_out) *xprev_out = xprev;
}

// ------------------------------------------------------------------ reverse

// Reverse one projection: given the adjoints of (x after, lam after) update
// them in place to the adjoints of (x before, lam before); accumulate the
// compliance and sphere adjoints.  x_before comes from the tape entry.
// Reverse of one membrane projection.  Forward: b = -C - at lam,
// J = G W G^T + at, J dl = b, lam' = lam + dl, x'_k = x_k + w_k G_k^T dl.
// alpha_bar: 3x3 adjoint of the compliance matrix alpha (= at h^2).
void reverse_membrane(const Ctx& c, const Row& r, const TapeEntry& te, double* xb, double* lamb, double* alpha_bar) {
  MemEval e;
  membrane_eval(c, r, te.x, e);
  const double* lam = te.lamv;
  double b[3], dl[3];
  for (int a = 0; a < 3; ++a) {
    b[a] = -e.C[a];
    for (int q = 0; q < 3; ++q) b[a] -= e.at[3 * a + q] * lam[q];
  }
  solve3(e.J, b, dl);
  double xbo[9];
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 3; ++a) xbo[3 * k + a] = xb[3 * r.v[k] + a];
  // through lam' = lam + dl and x' = x + W G^T dl
  double dlb[3];
  for (int q = 0; q < 3; ++q) {
    dlb[q] = lamb[r.lam + q];
    for (int i = 0; i < 9; ++i) dlb[q] += e.G[q][i] * e.w[i / 3] * xbo[i];
  }
  double Gb[3][9];
  for (int q = 0; q < 3; ++q)
    for (int i = 0; i < 9; ++i) Gb[q][i] = dl[q] * e.w[i / 3] * xbo[i];
  // J dl = b:  bbar = J^-T dlbar, Jbar = -bbar dl^T
  double Jt[9];
  for (int a = 0; a < 3; ++a) for (int q = 0; q < 3; ++q) Jt[3 * a + q] = e.J[3 * q + a];
  double bb[3];
  solve3(Jt, dlb, bb);
  double Jb[9];
  for (int a = 0; a < 3; ++a) for (int q = 0; q < 3; ++q) Jb[3 * a + q] = -bb[a] * dl[q];
  // J = G W G^T + at
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < 9; ++i) {
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) acc += (Jb[3 * a + q] + Jb[3 * q + a]) * e.G[q][i];
      Gb[a][i] += acc * e.w[i / 3];
    }
  const double h2 = c.h * c.h;
  for (int a = 0; a < 3; ++a)
    for (int q = 0; q < 3; ++q) alpha_bar[3 * a + q] += (Jb[3 * a + q] - bb[a] * lam[q]) / h2;
  // b = -C - at lam
  double Cb[3];
  for (int a = 0; a < 3; ++a) Cb[a] = -bb[a];
  for (int q = 0; q < 3; ++q) {
    double acc = lamb[r.lam + q];
    for (int a = 0; a < 3; ++a) acc -= e.at[3 * a + q] * bb[a];
    lamb[r.lam + q] = acc;
  }
  // x before: pass-through, plus C and G dependence (Hessian-vector products)
  Row rl = r;
  for (int k = 0; k < 3; ++k) rl.v[k] = k;
  for (int q = 0; q < 3; ++q) {
    rl.sub = q;
    double gdir[NG] = {0}, hv[NG];
    for (int i = 0; i < 9; ++i) gdir[i] = Gb[q][i];
    eval_hvp(&c.m, c.p, rl, te.x, gdir, hv);
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) xb[3 * r.v[k] + a] += Cb[q] * e.G[q][3 * k + a] + hv[3 * k + a];
  }
}

void reverse_row(const Ctx& c, const Row& r, const TapeEntry& te, double* xb, double* lamb,
                 double* alpha_bar_row, double* sphere_bar, double* gamma_bar) {
  const Scene* s = c.m.s;
  if (r.type == T_TRI) { reverse_membrane(c, r, te, xb, lamb, alpha_bar_row); return; }
  // rebuild a local position array holding only this row's vertices
  double xl[12];
  Row rl = r;
  for (int k = 0; k < r.nv; ++k) { rl.v[k] = k; for (int a = 0; a < 3; ++a) xl[3 * k + a] = te.x[3 * k + a]; }
  Eval e = eval_grad(&c.m, c.p, rl, xl);
  if (!e.ok) return;
  if (r.type == T_CONTACT && e.C >= 0.0) return;
  double at = row_compliance(&c.m, c.p, r) / (c.h * c.h);
  double w[4];
  double D = at;
  for (int k = 0; k < r.nv; ++k) {
    w[k] = s->inv_mass[r.v[k]];
    D += w[k] * (e.g[3 * k] * e.g[3 * k] + e.g[3 * k + 1] * e.g[3 * k + 1] + e.g[3 * k + 2] * e.g[3 * k + 2]);
  }
  if (D == 0.0) return;
  const double lb = te.lam;
  const double dl = (-e.C - at * lb) / D;
  // forward: lam' = lam + dl ;  x'_k = x_k + w_k dl gradC_k
  double dlb = lamb[r.lam];
  for (int k = 0; k < r.nv; ++k)
    for (int a = 0; a < 3; ++a) dlb += w[k] * e.g[3 * k + a] * xb[3 * r.v[k] + a];
  // adjoint of gradC_k (through the position update and through D)
  double gbar[NG] = {0};
  for (int k = 0; k < r.nv; ++k)
    for (int a = 0; a < 3; ++a)
      gbar[3 * k + a] = w[k] * dl * xb[3 * r.v[k] + a] - 2.0 * w[k] * e.g[3 * k + a] * dlb * dl / D;
  // dl = (-C - at lb)/D
  const double Cbar = -dlb / D;
  lamb[r.lam] = lamb[r.lam] - dlb * at / D;
  const double atbar = -dlb * (lb + dl) / D;
  *alpha_bar_row += atbar / (c.h * c.h);
  // x_before adjoint: x passes through; plus C and gradC dependence
  double hv[NG];
  eval_hvp(&c.m, c.p, rl, xl, gbar, hv);
  for (int k = 0; k < r.nv; ++k)
    for (int a = 0; a < 3; ++a) xb[3 * r.v[k] + a] += Cbar * e.g[3 * k + a] + hv[3 * k + a];
  if (r.type == T_CONTACT && sphere_bar) {
    for (int a = 0; a < 4; ++a) sphere_bar[a] += Cbar * e.g[12 + a] + hv[12 + a];
  }
  // C_H = det F - gamma: dC/dgamma = -1 (grad C does not depend on gamma)
  if (r.type == T_TET && r.sub == 1 && gamma_bar) *gamma_bar -= Cbar;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

typedef Scene orc_scene;
typedef Params orc_params;

// Rest data, exported so tests can inspect it.
int orc_rest_data(const orc_scene* s, double* L, double* theta0, double* B, double* vol) {
  Model m;
  if (build_model(s, &m)) return 1;
  if (L) std::copy(m.L.begin(), m.L.end(), L);
  if (theta0) std::copy(m.theta0.begin(), m.theta0.end(), theta0);
  if (B) std::copy(m.B.begin(), m.B.end(), B);
  if (vol) std::copy(m.vol.begin(), m.vol.end(), vol);
  return 0;
}

// Single-constraint evaluation for the unit tests: type 0..4, positions
// p[nv][3], rest data through `aux` (L; theta0; B[9] + gamma; tau; for a
// membrane Dm^-1[4] with sub = Voigt component),
// sphere[4] for contact.  Outputs C, grad[16] (positions then c, R) and,
// if gdir != null, hv[16] = Hessian * gdir.  Returns 0 if C is defined.
int orc_constraint(int type, int sub, const double* p, const double* aux, const double* sphere,
                   const double* gdir, double* C, double* grad, double* hv) {
  Scene s{};
  Model m;
  m.s = &s;
  Row r{}; r.type = type; r.sub = sub; r.item = 0;
  r.nv = type == T_DIST ? 2 : type == T_CONTACT ? 1 : type == T_TRI ? 3 : 4;
  for (int k = 0; k < r.nv; ++k) r.v[k] = k;
  m.L = {aux[0]};
  m.theta0 = {aux[0]};
  if (type == T_TET) { m.B.assign(aux, aux + 9); m.gamma = {aux[9]}; }
  if (type == T_TRI) m.tB.assign(aux, aux + 4);
  if (type == T_CONTACT) s.contact_thickness = aux[0];
  Params P{};
  if (sphere) for (int a = 0; a < 4; ++a) P.sphere[a] = sphere[a];
  Eval e = eval_grad(&m, &P, r, p);
  *C = e.C;
  if (grad) for (int i = 0; i < NG; ++i) grad[i] = e.g[i];
  if (gdir && hv) eval_hvp(&m, &P, r, p, gdir, hv);
  return e.ok ? 0 : 1;
}

// Squared distance from p[3] to the triangle tri[3][3] (the body pairing's
// distance), exported for the unit tests.
double orc_point_triangle_d2(const double* p, const double* tri) {
  return point_triangle_d2({p[0], p[1], p[2]}, {tri[0], tri[1], tri[2]}, {tri[3], tri[4], tri[5]},
                           {tri[6], tri[7], tri[8]});
}

// Forward rollout.  x_frames [F][V][3] receives the state at the end of
// each frame (may be null); x_final / v_final [V][3] the last state.
int orc_forward(const orc_scene* s, const orc_params* p, int F, const double* x0, const double* v0,
                double* x_frames, double* x_final, double* v_final) {
  Ctx c;
  if (build_model(s, &c.m)) return 1;
  set_materials(&c.m, p);
  c.p = p;
  c.h = s->dt / s->substeps;
  std::vector<int> pairv;
  if (s->n_body_tris > 0) {
    if (!p->body_x) return 1;
    c.pair = &pairv;
  }
  const int V = s->n_verts;
  std::vector<double> x(x0, x0 + 3 * (size_t)V), v(v0, v0 + 3 * (size_t)V), lam(c.m.n_lam, 0.0);
  for (int k = 0; k < V; ++k) {
    for (int a = 0; a < 3; ++a) { x[3 * k + a] = rnd(s, x[3 * k + a]); v[3 * k + a] = rnd(s, v[3 * k + a]); }
    if (s->inv_mass[k] == 0.0) for (int a = 0; a < 3; ++a) v[3 * k + a] = 0.0;
  }
  for (int f = 0; f < F; ++f) {
    const double* ff = p->f_ext ? p->f_ext + (size_t)f * 3 * V : nullptr;
    for (int st = 0; st < s->substeps; ++st) substep(c, x.data(), v.data(), lam.data(), ff, nullptr, nullptr);
    if (x_frames) std::copy(x.begin(), x.end(), x_frames + (size_t)f * 3 * V);
  }
  if (x_final) std::copy(x.begin(), x.end(), x_final);
  if (v_final) std::copy(v.begin(), v.end(), v_final);
  return 0;
}

// Exact adjoint (reverse through every substep, iteration and projection)
// of the rollout for the goal whose gradient with respect to the frame
// states is dLdx [F][V][3] (rows of frames not in the goal are zero) plus
// dLdv_final [V][3] (may be null).  Frames are recomputed from per-frame
// checkpoints.  Outputs (each may be null): g_x0, g_v0 [V][3], per-constraint
// compliance gradients, per-tet Young's modulus gradient, g_f [F][V][3],
// g_sphere [4] = (cx, cy, cz, R).
int orc_adjoint(const orc_scene* s, const orc_params* p, int F, const double* x0, const double* v0,
                const double* dLdx, const double* dLdv_final,
                double* g_x0, double* g_v0, double* g_dist_alpha, double* g_bend_alpha,
                double* g_tet_E, double* g_f, double* g_sphere, double* g_tet_mu, double* g_tet_lambda,
                double* g_tri_coef, double* g_body_x) {
  Ctx c;
  if (build_model(s, &c.m)) return 1;
  set_materials(&c.m, p);
  c.p = p;
  c.h = s->dt / s->substeps;
  std::vector<int> pairv;
  if (s->n_body_tris > 0) {
    if (!p->body_x) return 1;
    c.pair = &pairv;
  }
  const int V = s->n_verts;
  const size_t n3 = 3 * (size_t)V;
  // forward with per-frame checkpoints (state at the start of each frame)
  std::vector<double> x(x0, x0 + n3), v(v0, v0 + n3), lam(c.m.n_lam, 0.0);
  for (int k = 0; k < V; ++k) {
    for (int a = 0; a < 3; ++a) { x[3 * k + a] = rnd(s, x[3 * k + a]); v[3 * k + a] = rnd(s, v[3 * k + a]); }
    if (s->inv_mass[k] == 0.0) for (int a = 0; a < 3; ++a) v[3 * k + a] = 0.0;
  }
  std::vector<double> ck_x((size_t)F * n3), ck_v((size_t)F * n3);
  for (int f = 0; f < F; ++f) {
    std::copy(x.begin(), x.end(), ck_x.begin() + f * n3);
    std::copy(v.begin(), v.end(), ck_v.begin() + f * n3);
    const double* ff = p->f_ext ? p->f_ext + (size_t)f * n3 : nullptr;
    for (int st = 0; st < s->substeps; ++st) substep(c, x.data(), v.data(), lam.data(), ff, nullptr, nullptr);
  }
  // reverse
  std::vector<double> xb(n3, 0.0), vb(n3, 0.0), lamb(c.m.n_lam, 0.0);
  if (dLdv_final) std::copy(dLdv_final, dLdv_final + n3, vb.begin());
  std::vector<double> abar(c.m.n_lam, 0.0);   // per multiplier slot
  std::vector<double> gbar(s->n_tet, 0.0);     // per tet: dL/dgamma
  std::vector<double> tri_abar(9 * (size_t)s->n_tri, 0.0);   // per triangle: dL/dalpha (3x3)
  std::vector<double> body_bar(3 * (size_t)s->n_body_verts, 0.0);   // dL/dx_body
  double sph[4] = {0, 0, 0, 0};
  if (g_f) std::fill(g_f, g_f + (size_t)F * n3, 0.0);
  const double h = c.h;
  for (int f = F - 1; f >= 0; --f) {
    if (dLdx) for (size_t i = 0; i < n3; ++i) xb[i] += dLdx[(size_t)f * n3 + i];
    // recompute frame f, keeping the tape of every substep
    std::vector<double> xr(ck_x.begin() + f * n3, ck_x.begin() + (f + 1) * n3);
    std::vector<double> vr(ck_v.begin() + f * n3, ck_v.begin() + (f + 1) * n3);
    const double* ff = p->f_ext ? p->f_ext + (size_t)f * n3 : nullptr;
    std::vector<std::vector<TapeEntry>> tapes(s->substeps);
    for (int st = 0; st < s->substeps; ++st)
      substep(c, xr.data(), vr.data(), lam.data(), ff, &tapes[st], nullptr);
    for (int st = s->substeps - 1; st >= 0; --st) {
      // v' = (x'' - xprev)/h
      std::vector<double> xprev_bar(n3);
      for (size_t i = 0; i < n3; ++i) { xb[i] += vb[i] / h; xprev_bar[i] = -vb[i] / h; }
      std::fill(lamb.begin(), lamb.end(), 0.0);
      // sweeps in reverse
      const std::vector<TapeEntry>& tp = tapes[st];
      size_t per_iter = tp.size() / (s->iterations > 0 ? s->iterations : 1);
      for (int it = s->iterations - 1; it >= 0; --it) {
        size_t it_base = (size_t)it * per_iter;
        // walk sets backwards; offsets within the iteration
        std::vector<size_t> set_base(s->n_sets + 1, 0);
        for (int si = 0; si < s->n_sets; ++si)
          set_base[si + 1] = set_base[si] + (size_t)(s->set_off[si + 1] - s->set_off[si]) * set_rows(c.m, si);
        for (int si = s->n_sets - 1; si >= 0; --si) {
          int ty = s->set_type[si];
          int64_t b = s->set_off[si], e = s->set_off[si + 1];
          int nsub = set_rows(c.m, si);
          std::vector<double> sph_part((size_t)(e - b) * 4, 0.0);
          std::vector<double> body_part(ty == T_BODY ? (size_t)(e - b) * 9 : 0, 0.0);
#pragma omp parallel for schedule(static) num_threads(s->n_threads > 0 ? s->n_threads : 1)
          for (int64_t q = b; q < e; ++q) {
            for (int sub = nsub - 1; sub >= 0; --sub) {
              Row r = make_row(c.m, ty, s->set_items[q], sub);
              const TapeEntry& te = tp[it_base + set_base[si] + (size_t)(q - b) * nsub + sub];
              if (ty == T_BODY) {
                reverse_body(c, r.item, te, xb.data(), lamb.data(), &body_part[(q - b) * 9]);
                continue;
              }
              reverse_row(c, r, te, xb.data(), lamb.data(),
                          r.type == T_TRI ? &tri_abar[9 * (size_t)r.item] : &abar[r.lam], &sph_part[(q - b) * 4],
                          r.type == T_TET ? &gbar[r.item] : nullptr);
            }
          }
          if (ty == T_CONTACT)
            for (int64_t q = 0; q < e - b; ++q)
              for (int a = 0; a < 4; ++a) sph[a] += sph_part[q * 4 + a];
          if (ty == T_BODY)
            for (int64_t q = 0; q < e - b; ++q) {
              const TapeEntry& te = tp[it_base + set_base[si] + (size_t)q];
              if (te.tri < 0) continue;
              const int32_t* tv = s->body_tris + 3 * (int64_t)te.tri;
              for (int j = 0; j < 3; ++j)
                for (int a = 0; a < 3; ++a) body_bar[3 * (size_t)tv[j] + a] += body_part[q * 9 + 3 * j + a];
            }
        }
      }
      // predict: v' = v + h (g + w f) (free), x' = x + h v'
      for (int k = 0; k < V; ++k) {
        double w = s->inv_mass[k];
        for (int a = 0; a < 3; ++a) {
          size_t i = 3 * (size_t)k + a;
          double vmid_bar = w > 0.0 ? h * xb[i] : 0.0;
          if (g_f) g_f[(size_t)f * n3 + i] += h * w * vmid_bar;
          vb[i] = vmid_bar;
          xb[i] = xb[i] + xprev_bar[i];
        }
      }
    }
  }
  if (g_x0) std::copy(xb.begin(), xb.end(), g_x0);
  if (g_v0) std::copy(vb.begin(), vb.end(), g_v0);
  if (g_dist_alpha) for (int e = 0; e < s->n_dist; ++e) g_dist_alpha[e] = abar[c.m.lam_dist + e];
  if (g_bend_alpha) for (int e = 0; e < s->n_bend; ++e) g_bend_alpha[e] = abar[c.m.lam_bend + e];
  if (g_tet_E) {
    // alpha_D = 1/(mu V), alpha_H = 1/(lambda V) are both proportional to 1/E
    // at fixed nu, so d alpha / d E = -alpha / E.
    for (int t = 0; t < s->n_tet; ++t) {
      double aD = 1.0 / (c.m.mu[t] * c.m.vol[t]), aH = 1.0 / (c.m.lam[t] * c.m.vol[t]);
      double gd = abar[c.m.lam_tet + 2 * t], gh = abar[c.m.lam_tet + 2 * t + 1];
      g_tet_E[t] = -(gd * aD + gh * aH) / p->tet_E[t];
      // gamma = 1 + mu/lambda depends on nu only, not on E
    }
  }
  if (g_sphere) for (int a = 0; a < 4; ++a) g_sphere[a] = sph[a];
  // Lame parameters: alpha_D = 1/(mu V), alpha_H = 1/(lambda V),
  // gamma = 1 + mu/lambda (constant 1 with tet_gamma_one)
  for (int t = 0; t < s->n_tet && (g_tet_mu || g_tet_lambda); ++t) {
    double mu = c.m.mu[t], la = c.m.lam[t];
    double aD = 1.0 / (mu * c.m.vol[t]), aH = 1.0 / (la * c.m.vol[t]);
    double gd = abar[c.m.lam_tet + 2 * t], gh = abar[c.m.lam_tet + 2 * t + 1];
    double gg = s->tet_gamma_one ? 0.0 : gbar[t];
    if (g_tet_mu) g_tet_mu[t] = -gd * aD / mu + gg / la;
    if (g_tet_lambda) g_tet_lambda[t] = -gh * aH / la - gg * mu / (la * la);
  }
  if (g_body_x) std::copy(body_bar.begin(), body_bar.end(), g_body_x);
  // membrane coefficients: alpha = (A K)^-1, so d alpha = -alpha (A dK) alpha
  // and dL/dK = -A alpha^T alpha_bar alpha^T; K00 = C00, K01 = K10 = C01,
  // K11 = C11, K22 = C22
  for (int t = 0; t < s->n_tri && g_tri_coef; ++t) {
    double al[9], T1[9], Kb[9];
    membrane_alpha(c, t, al);
    const double* ab = &tri_abar[9 * (size_t)t];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += al[3 * k + i] * ab[3 * k + j];   // alpha^T alpha_bar
        T1[3 * i + j] = acc;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += T1[3 * i + k] * al[3 * j + k];   // ... alpha^T
        Kb[3 * i + j] = -c.m.tarea[t] * acc;
      }
    double* g = g_tri_coef + 4 * (size_t)t;
    g[0] = Kb[0];
    g[1] = Kb[1] + Kb[3];
    g[2] = Kb[4];
    g[3] = Kb[8];
  }
  return 0;
}

// Converged-limit (implicit) adjoint of Eq. adjointXPBD, one linear solve
// per substep, dense LU: for tiny meshes only.  Each substep's projection
// is treated as the implicit map x = y + M^-1 sum_j gradC_j lambda_j with
// lambda_j = -C_j / alpha~_j at the end-of-substep state (contacts active
// where C < 0 there).  Same outputs as orc_adjoint for the compliances of
// distance and bending rows, x0, v0 and f.
// pd != 0: each constraint's Hessian block -lambda_j Hess C_j is projected to
// positive semidefinite before assembly (Sec. 4.3, Positive Definite
// Projection; the rank-one block grad C grad C^T / alpha~ is already), so
// the system is symmetric positive definite.
// psd: with pd != 0, replaces the symmetric n x n matrix a (row-major) by its
// projection onto the positive semidefinite cone in place and returns 0; the
// caller supplies it (eigen-decomposition with negative eigenvalues dropped).
typedef int (*orc_psd_fn)(int n, double* a);
int orc_adjoint_implicit(const orc_scene* s, const orc_params* p, int F, const double* x0, const double* v0,
                         const double* dLdx, double* g_x0, double* g_v0, double* g_dist_alpha,
                         double* g_bend_alpha, double* g_f, int pd, orc_psd_fn psd) {
  if (pd && !psd) return 1;
  if (s->n_tri > 0 || s->n_body_tris > 0) return 2;   // membrane triangles: not part of the converged-limit cross-check
  Ctx c;
  if (build_model(s, &c.m)) return 1;
  set_materials(&c.m, p);
  c.p = p;
  c.h = s->dt / s->substeps;
  std::vector<int> pairv;
  if (s->n_body_tris > 0) {
    if (!p->body_x) return 1;
    c.pair = &pairv;
  }
  const int V = s->n_verts;
  const size_t n3 = 3 * (size_t)V;
  if (n3 > 1200) return 2;
  const int S = s->substeps;
  std::vector<double> x(x0, x0 + n3), v(v0, v0 + n3), lam(c.m.n_lam, 0.0);
  for (int k = 0; k < V; ++k)
    if (s->inv_mass[k] == 0.0) for (int a = 0; a < 3; ++a) v[3 * k + a] = 0.0;
  // forward keeping the end-of-substep positions
  std::vector<std::vector<double>> xend((size_t)F * S);
  for (int f = 0; f < F; ++f) {
    const double* ff = p->f_ext ? p->f_ext + (size_t)f * n3 : nullptr;
    for (int st = 0; st < S; ++st) {
      substep(c, x.data(), v.data(), lam.data(), ff, nullptr, nullptr);
      xend[(size_t)f * S + st] = x;
    }
  }
  std::vector<double> xb(n3, 0.0), vb(n3, 0.0), abar(c.m.n_lam, 0.0);
  if (g_f) std::fill(g_f, g_f + (size_t)F * n3, 0.0);
  const double h = c.h;
  std::vector<double> A(n3 * n3);
  for (int f = F - 1; f >= 0; --f) {
    if (dLdx) for (size_t i = 0; i < n3; ++i) xb[i] += dLdx[(size_t)f * n3 + i];
    for (int st = S - 1; st >= 0; --st) {
      const std::vector<double>& xe = xend[(size_t)f * S + st];
      std::vector<double> xprev_bar(n3);
      for (size_t i = 0; i < n3; ++i) { xb[i] += vb[i] / h; xprev_bar[i] = -vb[i] / h; }
      // K = sum_j (lambda_j Hess C_j - gradC_j gradC_j^T / at_j);  A = (I - M^-1 K)^T
      std::fill(A.begin(), A.end(), 0.0);
      for (size_t i = 0; i < n3; ++i) A[i * n3 + i] = 1.0;
      struct Act { Row r; Eval e; double at; };
      std::vector<Act> act;
      for (int si = 0; si < s->n_sets; ++si) {
        int ty = s->set_type[si];
        for (int64_t q = s->set_off[si]; q < s->set_off[si + 1]; ++q)
          for (int sub = 0; sub < set_rows(c.m, si); ++sub) {
            Row r = make_row(c.m, ty, s->set_items[q], sub);
            Eval e = eval_grad(&c.m, p, r, xe.data());
            if (!e.ok) continue;
            if (r.type == T_CONTACT && e.C >= 0.0) continue;
            double at = row_compliance(&c.m, p, r) / (h * h);
            if (at <= 0.0) return 3;
            act.push_back({r, e, at});
          }
      }
      for (const Act& a : act) {
        const Row& r = a.r;
        double lamj = -a.e.C / a.at;
        const int nl = 3 * r.nv;
        // local block N = -lambda Hess C, columns via HVPs with unit directions
        double N[NG * NG];
        for (int k2 = 0; k2 < r.nv; ++k2)
          for (int b2 = 0; b2 < 3; ++b2) {
            double dir[NG] = {0};
            dir[3 * k2 + b2] = 1.0;
            double hv[NG];
            eval_hvp(&c.m, p, r, xe.data(), dir, hv);
            for (int i = 0; i < nl; ++i) N[i * nl + 3 * k2 + b2] = -lamj * hv[i];
          }
        if (pd) {
          // symmetrise exactly, then project
          for (int i = 0; i < nl; ++i)
            for (int j = i + 1; j < nl; ++j) N[i * nl + j] = N[j * nl + i] = 0.5 * (N[i * nl + j] + N[j * nl + i]);
          if (psd(nl, N)) return 5;
        }
        for (int k2 = 0; k2 < r.nv; ++k2)
          for (int b2 = 0; b2 < 3; ++b2) {
            size_t col = 3 * (size_t)r.v[k2] + b2;
            for (int k1 = 0; k1 < r.nv; ++k1)
              for (int b1 = 0; b1 < 3; ++b1) {
                size_t row = 3 * (size_t)r.v[k1] + b1;
                // K = lambda Hess C - grad C grad C^T / alpha~ = -(N + g g^T / alpha~)
                double Kv = -N[(3 * k1 + b1) * nl + 3 * k2 + b2] - a.e.g[3 * k1 + b1] * a.e.g[3 * k2 + b2] / a.at;
                double w = s->inv_mass[r.v[k1]];
                // (I - M^-1 K): entry (row, col) ; we store the transpose
                A[col * n3 + row] -= w * Kv;
              }
          }
      }
      // solve A wv = xb (dense LU with partial pivoting)
      std::vector<double> M(A), rhs(xb);
      std::vector<int> piv(n3);
      for (size_t k = 0; k < n3; ++k) {
        size_t pr = k; double best = std::fabs(M[k * n3 + k]);
        for (size_t i = k + 1; i < n3; ++i) if (std::fabs(M[i * n3 + k]) > best) { best = std::fabs(M[i * n3 + k]); pr = i; }
        if (best == 0.0) return 4;
        if (pr != k) { for (size_t j = 0; j < n3; ++j) std::swap(M[k * n3 + j], M[pr * n3 + j]); std::swap(rhs[k], rhs[pr]); }
        for (size_t i = k + 1; i < n3; ++i) {
          double l = M[i * n3 + k] / M[k * n3 + k];
          if (l == 0.0) continue;
          for (size_t j = k; j < n3; ++j) M[i * n3 + j] -= l * M[k * n3 + j];
          rhs[i] -= l * rhs[k];
        }
      }
      std::vector<double> wv(n3);
      for (size_t k = n3; k-- > 0;) {
        double acc = rhs[k];
        for (size_t j = k + 1; j < n3; ++j) acc -= M[k * n3 + j] * wv[j];
        wv[k] = acc / M[k * n3 + k];
      }
      // compliance adjoints: d x / d at_j = M^-1 gradC_j d lambda_j / d at_j,
      // d lambda_j / d at_j = C_j / at_j^2 = -lambda_j / at_j
      for (const Act& a : act) {
        const Row& r = a.r;
        double lamj = -a.e.C / a.at;
        double acc = 0.0;
        for (int k = 0; k < r.nv; ++k) {
          double w = s->inv_mass[r.v[k]];
          for (int b = 0; b < 3; ++b) acc += wv[3 * (size_t)r.v[k] + b] * w * a.e.g[3 * k + b];
        }
        abar[r.lam] += acc * (-lamj / a.at) / (h * h);
      }
      for (int k = 0; k < V; ++k) {
        double w = s->inv_mass[k];
        for (int a = 0; a < 3; ++a) {
          size_t i = 3 * (size_t)k + a;
          double vmid_bar = w > 0.0 ? h * wv[i] : 0.0;
          if (g_f) g_f[(size_t)f * n3 + i] += h * w * vmid_bar;
          vb[i] = vmid_bar;
          xb[i] = wv[i] + xprev_bar[i];
        }
      }
    }
  }
  if (g_x0) std::copy(xb.begin(), xb.end(), g_x0);
  if (g_v0) std::copy(vb.begin(), vb.end(), g_v0);
  if (g_dist_alpha) for (int e = 0; e < s->n_dist; ++e) g_dist_alpha[e] = abar[c.m.lam_dist + e];
  if (g_bend_alpha) for (int e = 0; e < s->n_bend; ++e) g_bend_alpha[e] = abar[c.m.lam_bend + e];
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
