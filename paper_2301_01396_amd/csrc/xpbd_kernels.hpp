// HIP kernels of the XPBD forward sweeps and their exact adjoint (gfx950).
//
// One thread owns one constraint of an independent set, so the sets need
// no atomics: vertex state is gathered and scattered as 16-byte (FP32) or
// 32-byte (FP64) packed records {x, y, z, w} with w the inverse mass, and
// the vertex adjoints as {xbar, ybar, zbar, w}.  Constraint records are
// structure-of-arrays in schedule order, so every record load is coalesced.
//
// Forward items can record, per projection, exactly the inputs its adjoint
// needs (the vertex differences and the multiplier before the update);
// reverse items recompute C, grad C, D and dlambda from that record bit for
// bit and apply the chain rule to
//     dlambda = (-C - at lambda) / D,  lambda += dlambda,
//     x_k += w_k dlambda grad_k C
// (Eq. xpbd and the position update of Sec. 3.1), with the partials of
// Sec. 4.3: the adjoint of grad C (through the position update and through
// D = sum_k w_k |grad_k C|^2 + at), the Hessian-vector product it feeds,
// and the compliance adjoint -dlbar (lambda + dlambda) / D.
//
// Each per-item body is a device function used twice: by a plain kernel
// (one launch per independent set) and by the persistent program kernel,
// which walks a list of phases (sets, per-vertex steps) inside one
// cooperative launch with a grid-wide barrier between phases.
#pragma once
#include "xpbd_device.hpp"

namespace xpbd {

constexpr int kBlock = 256;
// per-set kernels accept any power-of-two workgroup size up to this
// (chosen per context; every size computes the same result)
constexpr int kMaxBlock = 1024;
// bytes of each device copy of the per-set kernels' parameter block (Dev)
constexpr size_t kDevBlk = 1024;

template <class T> struct TetRec {
  const int4* idx;
  const T* B;        // [9][n_tet] Dm^-1 row-major entries
  const T* atD;      // [n_tet] alpha_D / h^2
  const T* atH;      // [n_tet] alpha_H / h^2
  const T* gamma;    // [n_tet]
  int n;             // n_tet (stride of B)
};

template <class T> struct Sphere { T cx, cy, cz, R, tau, at; };

// Membrane triangles (orthotropic StVK, Sec. 5.1): Dm^-1 and the nonzero
// entries of at = alpha / h^2 (alpha = (A K)^-1 is block diagonal: a 2x2
// warp/weft block and the shear entry), SoA in internal order.
template <class T> struct TriRec {
  const int4* idx;   // v0, v1, v2, unused
  const T* B;        // [4][n] Dm^-1 row-major (B00, B01, B10, B11)
  const T* at;       // [4][n] at00, at01, at11, at22
  int n;
};

// Every device array and scalar the sweeps use (passed by value).
template <class T> struct Dev {
  Vec4<T>* X;    // positions + inverse mass
  Vec4<T>* Vv;   // velocities
  Vec4<T>* Xp;   // positions at the start of the substep
  Vec4<T>* XB;   // position adjoints + inverse mass
  Vec4<T>* VB;   // velocity adjoints
  int V;
  const int2* d_idx; const T* d_rest; const T* d_at; T* d_lam; T* d_lamb; T* d_ab; double* d_acc;
  const int4* b_idx; const T* b_th0; const T* b_at; T* b_lam; T* b_lamb; T* b_ab; double* b_acc;
  TetRec<T> tr; T* t_lamD; T* t_lamH; T* t_lambD; T* t_lambH; T* t_eb; double* t_acc;
  const int* c_vid; T* c_lam; T* c_lamb; Vec4<T>* c_sacc; const int* c_order;
  TriRec<T> mr; T* m_lam; T* m_lamb; T* m_ab; double* m_acc;   // lam, lamb [3][n]; ab, acc [4][n]
  // body collider: contact items (cloth vertex, multiplier, its adjoint), the
  // substep's pairing (body triangle per item, -1 none), body vertices
  // [n_bv][3], triangles, FP64 body-vertex gradient (null: not wanted)
  const int* bc_vid; T* bc_lam; T* bc_lamb; const int* bpair; const T* bx; const int4* btri; double* bgrad;
  T bc_tau, bc_at;
  Sphere<T> sph;
  T h, inv_h, gx, gy, gz;
};

// ===================================================================== projection cores
// Each core works on register copies of one constraint's vertices and
// record, so the same arithmetic serves vertex state in global memory and
// vertex tiles in LDS.  Forward cores return lambda after the projection
// (lambda before when it is skipped), set `moved` when the projection was
// applied (its vertex copies then hold x + w dlambda grad C and must be
// stored, even where dlambda vanished when added to lambda) and optionally
// emit the adjoint's record; reverse cores update the vertex adjoints,
// lambda_bar and the compliance adjoint in place.

template <class T, bool TAPE>
__device__ __forceinline__ T dist_fwd(Vec4<T>& a, Vec4<T>& b, T rest, T a_t, T lb, Vec4<T>* tape, bool& moved) {
  V3<T> r = xyz(a) - xyz(b);
  if (TAPE) *tape = Vec4<T>{r.x, r.y, r.z, lb};
  DistEval<T> ev = dist_eval(r, rest);
  T Dn = a.w + b.w + a_t;
  moved = ev.ok && Dn > T(0);
  if (!moved) return lb;
  T dl = (-ev.C - a_t * lb) / Dn;
  T sa = a.w * dl, sb = b.w * dl;
  a.x += sa * ev.n.x; a.y += sa * ev.n.y; a.z += sa * ev.n.z;
  b.x -= sb * ev.n.x; b.y -= sb * ev.n.y; b.z -= sb * ev.n.z;
  return lb + dl;
}

// bending record of set item t: Vec4 (e, lambda) at tape[t], Vec4 (a, b.x) at
// tape[count + t], Vec2 (b.y, b.z) at element t of the Vec2 array that
// starts at tape + 2 * count
template <class T, bool TAPE>
__device__ __forceinline__ T bend_fwd(Vec4<T> p[4], T theta0, T a_t, T lb, Vec4<T>* tape, int t, int count,
                                      bool& moved) {
  V3<T> e = xyz(p[1]) - xyz(p[0]), a = xyz(p[2]) - xyz(p[0]), b = xyz(p[3]) - xyz(p[0]);
  if (TAPE) {
    tape[t] = Vec4<T>{e.x, e.y, e.z, lb};
    tape[count + t] = Vec4<T>{a.x, a.y, a.z, b.x};
    reinterpret_cast<Vec2<T>*>(tape + 2 * count)[t] = Vec2<T>{b.y, b.z};
  }
  BendEval<T> ev = bend_eval(e, a, b, theta0);
  T Dn = a_t;
#pragma unroll
  for (int k = 0; k < 4; ++k) Dn += p[k].w * dot(ev.g[k], ev.g[k]);
  moved = ev.ok && Dn > T(0);
  if (!moved) return lb;
  T dl = (-ev.C - a_t * lb) / Dn;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T s = p[k].w * dl;
    p[k].x += s * ev.g[k].x; p[k].y += s * ev.g[k].y; p[k].z += s * ev.g[k].z;
  }
  return lb + dl;
}

template <class T> __device__ __forceinline__ M3<T> load_B(const T* B, int n, int j) {
  M3<T> m;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) m.m[r][c] = B[(size_t)(r * 3 + c) * n + j];
  return m;
}

// One tet item = deviatoric projection then hydrostatic projection.  The
// hydrostatic constraint is evaluated on the edge matrix updated in place by
// the deviatoric correction (d_k += delta_k - delta_0).
template <class T> struct TetStep {
  TetEval<T> evD, evH;
  bool appD, appH;
  T DD, DH, dlD, dlH;
  V3<T> dD[4], dH[4];     // position corrections of each projection
};
template <class T>
__device__ __forceinline__ void tet_step(const V3<T> d0[3], const T w[4], const M3<T>& B, T atD, T atH, T gamma,
                                         T lD, T lH, TetStep<T>& s) {
  s.evD = tet_dev_eval(d0, B);
  s.DD = atD;
#pragma unroll
  for (int k = 0; k < 4; ++k) s.DD += w[k] * dot(s.evD.g[k], s.evD.g[k]);
  s.appD = s.evD.ok && s.DD > T(0);
  s.dlD = s.appD ? (-s.evD.C - atD * lD) / s.DD : T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) s.dD[k] = s.appD ? (w[k] * s.dlD) * s.evD.g[k] : V3<T>{T(0), T(0), T(0)};
  V3<T> d1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) d1[c] = d0[c] + (s.dD[c + 1] - s.dD[0]);
  s.evH = tet_hyd_eval(d1, B, gamma);
  s.DH = atH;
#pragma unroll
  for (int k = 0; k < 4; ++k) s.DH += w[k] * dot(s.evH.g[k], s.evH.g[k]);
  s.appH = s.DH > T(0);
  s.dlH = s.appH ? (-s.evH.C - atH * lH) / s.DH : T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) s.dH[k] = s.appH ? (w[k] * s.dlH) * s.evH.g[k] : V3<T>{T(0), T(0), T(0)};
}

template <class T, bool TAPE>
__device__ __forceinline__ void tet_fwd(Vec4<T> p[4], const M3<T>& B, T atD, T atH, T gamma, T& lD, T& lH,
                                        Vec4<T>* tape, int count) {
  V3<T> d[3] = {xyz(p[1]) - xyz(p[0]), xyz(p[2]) - xyz(p[0]), xyz(p[3]) - xyz(p[0])};
  if (TAPE) {
    tape[0] = Vec4<T>{d[0].x, d[0].y, d[0].z, d[1].x};
    tape[count] = Vec4<T>{d[1].y, d[1].z, d[2].x, d[2].y};
    tape[2 * count] = Vec4<T>{d[2].z, lD, lH, T(0)};
  }
  T w[4] = {p[0].w, p[1].w, p[2].w, p[3].w};
  TetStep<T> s;
  tet_step(d, w, B, atD, atH, gamma, lD, lH, s);
  lD = lD + s.dlD;
  lH = lH + s.dlH;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    p[k].x = (p[k].x + s.dD[k].x) + s.dH[k].x;
    p[k].y = (p[k].y + s.dD[k].y) + s.dH[k].y;
    p[k].z = (p[k].z + s.dD[k].z) + s.dH[k].z;
  }
}

template <class T, bool TAPE>
__device__ __forceinline__ T contact_fwd(Vec4<T>& p, const Sphere<T>& S, T lb, Vec4<T>* tape, bool& moved) {
  if (TAPE) *tape = Vec4<T>{p.x, p.y, p.z, lb};
  ContactEval<T> ev = contact_eval(V3<T>{p.x - S.cx, p.y - S.cy, p.z - S.cz}, S.R, S.tau);
  T Dn = p.w + S.at;
  moved = ev.ok && ev.C < T(0) && Dn > T(0);
  if (!moved) return lb;
  T dl = (-ev.C - S.at * lb) / Dn;
  T s = p.w * dl;
  p.x += s * ev.n.x; p.y += s * ev.n.y; p.z += s * ev.n.z;
  return lb + dl;
}

// ---- membrane triangle: one vector projection of C = (E_uu, E_vv, 2 E_uv)
// With F = [d1 d2] Dm^-1 = [fu fv] the constraint depends on x only through
// fu = sum_k bu_k x_k and fv = sum_k bv_k x_k (bu, bv: the columns of
// Dm^-1 spread over the corners, each summing to zero), so
//   grad_k C_uu = bu_k fu,  grad_k C_vv = bv_k fv,  grad_k C_uv = bu_k fv + bv_k fu,
// and with S_ab = sum_k w_k a_k b_k the system J = grad C W grad C^T + at is
//   J00 = Suu P, J11 = Svv Q, J01 = Suv R, J02 = Suu R + Suv P,
//   J12 = Suv Q + Svv R, J22 = Suu Q + 2 Suv R + Svv P   (+ at),
// P = |fu|^2, Q = |fv|^2, R = fu . fv.
template <class T> struct TriStep {
  V3<T> fu, fv;
  T bu[3], bv[3];
  T Suu, Svv, Suv, P, Q, R;
  T Ji[6];      // J^-1: 00 01 02 11 12 22
  T dl[3];
  bool ok;
};
template <class T>
__device__ __forceinline__ void tri_step(V3<T> d1, V3<T> d2, const T w[3], const T B[4], const T at[4],
                                         const T lam[3], TriStep<T>& s) {
  s.fu = B[0] * d1 + B[2] * d2;
  s.fv = B[1] * d1 + B[3] * d2;
  s.bu[0] = -(B[0] + B[2]); s.bu[1] = B[0]; s.bu[2] = B[2];
  s.bv[0] = -(B[1] + B[3]); s.bv[1] = B[1]; s.bv[2] = B[3];
  s.Suu = T(0); s.Svv = T(0); s.Suv = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.Suu += w[k] * s.bu[k] * s.bu[k];
    s.Svv += w[k] * s.bv[k] * s.bv[k];
    s.Suv += w[k] * s.bu[k] * s.bv[k];
  }
  s.P = dot(s.fu, s.fu); s.Q = dot(s.fv, s.fv); s.R = dot(s.fu, s.fv);
  const T J00 = s.Suu * s.P + at[0], J11 = s.Svv * s.Q + at[2];
  const T J22 = s.Suu * s.Q + T(2) * s.Suv * s.R + s.Svv * s.P + at[3];
  const T J01 = s.Suv * s.R + at[1], J02 = s.Suu * s.R + s.Suv * s.P, J12 = s.Suv * s.Q + s.Svv * s.R;
  // symmetric inverse by cofactors
  const T c00 = J11 * J22 - J12 * J12, c01 = J02 * J12 - J01 * J22, c02 = J01 * J12 - J02 * J11;
  const T c11 = J00 * J22 - J02 * J02, c12 = J01 * J02 - J00 * J12, c22 = J00 * J11 - J01 * J01;
  const T det = J00 * c00 + J01 * c01 + J02 * c02;
  s.ok = det > T(0);
  const T id = s.ok ? T(1) / det : T(0);
  s.Ji[0] = c00 * id; s.Ji[1] = c01 * id; s.Ji[2] = c02 * id;
  s.Ji[3] = c11 * id; s.Ji[4] = c12 * id; s.Ji[5] = c22 * id;
  // b = -C - at lam  (at has no 02 / 12 entries)
  const T b0 = -(T(0.5) * (s.P - T(1))) - (at[0] * lam[0] + at[1] * lam[1]);
  const T b1 = -(T(0.5) * (s.Q - T(1))) - (at[1] * lam[0] + at[2] * lam[1]);
  const T b2 = -s.R - at[3] * lam[2];
  s.dl[0] = s.Ji[0] * b0 + s.Ji[1] * b1 + s.Ji[2] * b2;
  s.dl[1] = s.Ji[1] * b0 + s.Ji[3] * b1 + s.Ji[4] * b2;
  s.dl[2] = s.Ji[2] * b0 + s.Ji[4] * b1 + s.Ji[5] * b2;
}

// record of set item t: Vec4 (d1, d2.x) at tape[t], (d2.y, d2.z, lam0, lam1)
// at tape[count + t], (lam2, 0, 0, 0) at tape[2 count + t]
template <class T, bool TAPE>
__device__ __forceinline__ bool tri_fwd(Vec4<T> p[3], const T B[4], const T at[4], T lam[3], Vec4<T>* tape, int t,
                                        int count) {
  V3<T> d1 = xyz(p[1]) - xyz(p[0]), d2 = xyz(p[2]) - xyz(p[0]);
  if (TAPE) {
    tape[t] = Vec4<T>{d1.x, d1.y, d1.z, d2.x};
    tape[count + t] = Vec4<T>{d2.y, d2.z, lam[0], lam[1]};
    tape[2 * count + t] = Vec4<T>{lam[2], T(0), T(0), T(0)};
  }
  T w[3] = {p[0].w, p[1].w, p[2].w};
  TriStep<T> s;
  tri_step(d1, d2, w, B, at, lam, s);
  if (!s.ok) return false;
#pragma unroll
  for (int c = 0; c < 3; ++c) lam[c] = lam[c] + s.dl[c];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T a = w[k] * (s.bu[k] * s.dl[0] + s.bv[k] * s.dl[2]);
    const T b = w[k] * (s.bv[k] * s.dl[1] + s.bu[k] * s.dl[2]);
    p[k].x += a * s.fu.x + b * s.fv.x;
    p[k].y += a * s.fu.y + b * s.fv.y;
    p[k].z += a * s.fu.z + b * s.fv.z;
  }
  return true;
}

// Adjoint of one projection given the adjoints of its outputs: gradient g_k,
// weights w_k, iD = 1 / D (the denominator's reciprocal), dlambda,
// lambda_bar, position adjoints xb_k.  Returns dlambda_bar; writes gbar_k
// (adjoint of grad_k C).  The reverse cores divide by D once (iD) and
// multiply: the adjoint needs no quotient that the forward also forms (only
// dlambda must repeat the forward's division exactly, and it does), and the
// kernels spend most of their issue slots on VALU arithmetic.
template <class T, int N>
__device__ __forceinline__ T proj_adjoint(const V3<T> g[N], const T w[N], T iD, T dl, T lbar, const V3<T> xb[N],
                                          V3<T> gb[N]) {
  T dlb = lbar;
#pragma unroll
  for (int k = 0; k < N; ++k) dlb += w[k] * dot(g[k], xb[k]);
  T c = T(2) * dlb * dl * iD;
#pragma unroll
  for (int k = 0; k < N; ++k) gb[k] = {w[k] * (dl * xb[k].x - c * g[k].x), w[k] * (dl * xb[k].y - c * g[k].y),
                                      w[k] * (dl * xb[k].z - c * g[k].z)};
  return dlb;
}

// A and Bv hold (xbar, w) of the two vertices; returns true if they changed.
template <class T>
__device__ __forceinline__ bool dist_rev(Vec4<T>& A, Vec4<T>& Bv, Vec4<T> tp, T rest, T a_t, T& lbar, T& ab) {
  DistEval<T> ev = dist_eval(V3<T>{tp.x, tp.y, tp.z}, rest);
  T Dn = A.w + Bv.w + a_t;
  if (!(ev.ok && Dn > T(0))) return false;
  T lb = tp.w;
  T dl = (-ev.C - a_t * lb) / Dn;
  const T iD = T(1) / Dn;
  V3<T> xa = xyz(A), xb = xyz(Bv);
  T dlb = lbar + A.w * dot(ev.n, xa) - Bv.w * dot(ev.n, xb);
  // Hessian of |r| is P / |r| (P = I - n n^T); the D-path part of gbar is
  // along n and vanishes under P, leaving dl * P (w_i xa - w_j xb) / |r|.
  V3<T> u = A.w * xa - Bv.w * xb;
  T un = dot(ev.n, u);
  T s = dl * ev.inv;
  V3<T> hv = {s * (u.x - un * ev.n.x), s * (u.y - un * ev.n.y), s * (u.z - un * ev.n.z)};
  T Cb = -dlb * iD;
  lbar = lbar - dlb * a_t * iD;
  ab = ab - dlb * (lb + dl) * iD;
  A.x += Cb * ev.n.x + hv.x; A.y += Cb * ev.n.y + hv.y; A.z += Cb * ev.n.z + hv.z;
  Bv.x -= Cb * ev.n.x + hv.x; Bv.y -= Cb * ev.n.y + hv.y; Bv.z -= Cb * ev.n.z + hv.z;
  return true;
}

template <class T>
__device__ __forceinline__ bool bend_rev(Vec4<T> P[4], const Vec4<T>* tape, int t, int count, T theta0, T a_t,
                                         T& lbar, T& ab) {
  Vec4<T> tA = tape[t], tB = tape[count + t];
  Vec2<T> tC = reinterpret_cast<const Vec2<T>*>(tape + 2 * count)[t];
  V3<T> e = {tA.x, tA.y, tA.z}, a = {tB.x, tB.y, tB.z}, b = {tB.w, tC.x, tC.y};
  T lb = tA.w;
  BendEval<T> ev = bend_eval(e, a, b, theta0);
  T w[4] = {P[0].w, P[1].w, P[2].w, P[3].w};
  T Dn = a_t;
#pragma unroll
  for (int k = 0; k < 4; ++k) Dn += w[k] * dot(ev.g[k], ev.g[k]);
  if (!(ev.ok && Dn > T(0))) return false;
  T dl = (-ev.C - a_t * lb) / Dn;
  const T iD = T(1) / Dn;
  V3<T> xb[4] = {xyz(P[0]), xyz(P[1]), xyz(P[2]), xyz(P[3])};
  V3<T> gb[4], hv[4];
  T dlb = proj_adjoint<T, 4>(ev.g, w, iD, dl, lbar, xb, gb);
  bend_hvp(e, a, b, gb, hv);
  T Cb = -dlb * iD;
  lbar = lbar - dlb * a_t * iD;
  ab = ab - dlb * (lb + dl) * iD;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    P[k].x += Cb * ev.g[k].x + hv[k].x;
    P[k].y += Cb * ev.g[k].y + hv[k].y;
    P[k].z += Cb * ev.g[k].z + hv[k].z;
  }
  return true;
}

// tet: ebar accumulates sum over projections of (atbar_D at_D + atbar_H at_H),
// i.e. alphabar_D alpha_D + alphabar_H alpha_H, whence dL/dE = -ebar / E.
template <class T>
// ebD, ebH accumulate abar~ alpha~ of the deviatoric and hydrostatic rows (the
// compliance adjoints times the compliances), gb the adjoint of gamma
// (C_H = det F - gamma, so gbar -= Cbar_H)
__device__ __forceinline__ bool tet_rev(Vec4<T> P[4], const Vec4<T>* tape, int count, const M3<T>& B, T atD, T atH,
                                        T gamma, T& lbD, T& lbH, T& ebD, T& ebH, T& gmb) {
  Vec4<T> t0 = tape[0], t1 = tape[count], t2 = tape[2 * count];
  V3<T> d[3] = {{t0.x, t0.y, t0.z}, {t0.w, t1.x, t1.y}, {t1.z, t1.w, t2.x}};
  T lD = t2.y, lH = t2.z;
  T w[4] = {P[0].w, P[1].w, P[2].w, P[3].w};
  TetStep<T> s;
  tet_step(d, w, B, atD, atH, gamma, lD, lH, s);
  V3<T> xb[4] = {xyz(P[0]), xyz(P[1]), xyz(P[2]), xyz(P[3])};
  V3<T> gb[4], hv[4];
  if (s.appH) {
    const T iD = T(1) / s.DH;
    T dlb = proj_adjoint<T, 4>(s.evH.g, w, iD, s.dlH, lbH, xb, gb);
    tet_hyd_hvp(s.evH, B, gb, hv);
    T Cb = -dlb * iD;
    lbH = lbH - dlb * atH * iD;
    ebH = ebH - dlb * (lH + s.dlH) * iD * atH;
    gmb = gmb - Cb;
#pragma unroll
    for (int k = 0; k < 4; ++k) xb[k] = xb[k] + (Cb * s.evH.g[k] + hv[k]);
  }
  if (s.appD) {
    const T iD = T(1) / s.DD;
    T dlb = proj_adjoint<T, 4>(s.evD.g, w, iD, s.dlD, lbD, xb, gb);
    tet_dev_hvp(s.evD, B, gb, hv);
    T Cb = -dlb * iD;
    lbD = lbD - dlb * atD * iD;
    ebD = ebD - dlb * (lD + s.dlD) * iD * atD;
#pragma unroll
    for (int k = 0; k < 4; ++k) xb[k] = xb[k] + (Cb * s.evD.g[k] + hv[k]);
  }
  if (!(s.appD || s.appH)) return false;
#pragma unroll
  for (int k = 0; k < 4; ++k) { P[k].x = xb[k].x; P[k].y = xb[k].y; P[k].z = xb[k].z; }
  return true;
}

// contact: also accumulates the sphere adjoint (cbar, Rbar) in sa
template <class T>
__device__ __forceinline__ bool contact_rev(Vec4<T>& P, Vec4<T> tp, const Sphere<T>& S, T& lbar, Vec4<T>& sa) {
  ContactEval<T> ev = contact_eval(V3<T>{tp.x - S.cx, tp.y - S.cy, tp.z - S.cz}, S.R, S.tau);
  T Dn = P.w + S.at;
  if (!(ev.ok && ev.C < T(0) && Dn > T(0))) return false;
  T lb = tp.w;
  T dl = (-ev.C - S.at * lb) / Dn;
  const T iD = T(1) / Dn;
  V3<T> xb = xyz(P);
  T dlb = lbar + P.w * dot(ev.n, xb);
  T c = T(2) * dlb * dl * iD;
  V3<T> gb = {P.w * (dl * xb.x - c * ev.n.x), P.w * (dl * xb.y - c * ev.n.y), P.w * (dl * xb.z - c * ev.n.z)};
  T gn = dot(ev.n, gb);
  T inv = T(1) / ev.d;
  V3<T> hv = {inv * (gb.x - gn * ev.n.x), inv * (gb.y - gn * ev.n.y), inv * (gb.z - gn * ev.n.z)};
  T Cb = -dlb * iD;
  lbar = lbar - dlb * S.at * iD;
  P.x += Cb * ev.n.x + hv.x; P.y += Cb * ev.n.y + hv.y; P.z += Cb * ev.n.z + hv.z;
  // C = |x - c| - R - tau: dC/dc = -n, dC/dR = -1, d(grad_x C)/dc = -P/|x-c|
  sa.x -= Cb * ev.n.x + hv.x; sa.y -= Cb * ev.n.y + hv.y; sa.z -= Cb * ev.n.z + hv.z;
  sa.w -= Cb;
  return true;
}

// Reverse of one membrane projection.  From the adjoints xbar_k of the
// corrected positions and lbar of the multipliers after it:
//   dlbar = lbar + grad C W xbar,  bbar = J^-1 dlbar,  Cbar = -bbar,
//   lbar <- lbar - at bbar,  Jbar = -bbar dl^T,  atbar += -bbar (lam + dl)^T,
// and the adjoints of fu, fv collect the position update's dependence on
// them, J's (through P, Q, R) and C's, then spread to the corners with bu,
// bv.  ab accumulates the symmetric part of atbar: (00, 01 + 10, 11, 22).
template <class T>
__device__ __forceinline__ bool tri_rev(Vec4<T> P[3], const Vec4<T>* tape, int t, int count, const T B[4],
                                        const T at[4], T lbar[3], T ab[4]) {
  Vec4<T> t0 = tape[t], t1 = tape[count + t], t2 = tape[2 * count + t];
  V3<T> d1 = {t0.x, t0.y, t0.z}, d2 = {t0.w, t1.x, t1.y};
  T lam[3] = {t1.z, t1.w, t2.x};
  T w[3] = {P[0].w, P[1].w, P[2].w};
  TriStep<T> s;
  tri_step(d1, d2, w, B, at, lam, s);
  if (!s.ok) return false;
  V3<T> xb[3] = {xyz(P[0]), xyz(P[1]), xyz(P[2])};
  T pu[3], pv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { pu[k] = dot(s.fu, xb[k]); pv[k] = dot(s.fv, xb[k]); }
  T dlb0 = lbar[0], dlb1 = lbar[1], dlb2 = lbar[2];
  V3<T> fub = {T(0), T(0), T(0)}, fvb = {T(0), T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dlb0 += w[k] * s.bu[k] * pu[k];
    dlb1 += w[k] * s.bv[k] * pv[k];
    dlb2 += w[k] * (s.bv[k] * pu[k] + s.bu[k] * pv[k]);
    const T a = w[k] * (s.bu[k] * s.dl[0] + s.bv[k] * s.dl[2]);
    const T b = w[k] * (s.bv[k] * s.dl[1] + s.bu[k] * s.dl[2]);
    fub = fub + a * xb[k];
    fvb = fvb + b * xb[k];
  }
  const T bb0 = s.Ji[0] * dlb0 + s.Ji[1] * dlb1 + s.Ji[2] * dlb2;
  const T bb1 = s.Ji[1] * dlb0 + s.Ji[3] * dlb1 + s.Ji[4] * dlb2;
  const T bb2 = s.Ji[2] * dlb0 + s.Ji[4] * dlb1 + s.Ji[5] * dlb2;
  const T ln0 = lam[0] + s.dl[0], ln1 = lam[1] + s.dl[1], ln2 = lam[2] + s.dl[2];
  lbar[0] = lbar[0] - (at[0] * bb0 + at[1] * bb1);
  lbar[1] = lbar[1] - (at[1] * bb0 + at[2] * bb1);
  lbar[2] = lbar[2] - at[3] * bb2;
  ab[0] -= bb0 * ln0;
  ab[1] -= bb0 * ln1 + bb1 * ln0;
  ab[2] -= bb1 * ln1;
  ab[3] -= bb2 * ln2;
  // J's weights: M_cc = Jbar_cc, M_cd = Jbar_cd + Jbar_dc (c < d), Jbar = -bbar dl^T
  const T M00 = -bb0 * s.dl[0], M11 = -bb1 * s.dl[1], M22 = -bb2 * s.dl[2];
  const T M01 = -(bb0 * s.dl[1] + bb1 * s.dl[0]), M02 = -(bb0 * s.dl[2] + bb2 * s.dl[0]);
  const T M12 = -(bb1 * s.dl[2] + bb2 * s.dl[1]);
  // adjoints of P, Q, R through J, plus C = (P/2 - 1/2, Q/2 - 1/2, R) with Cbar = -bbar
  const T Pb = M00 * s.Suu + M02 * s.Suv + M22 * s.Svv - T(0.5) * bb0;
  const T Qb = M11 * s.Svv + M12 * s.Suv + M22 * s.Suu - T(0.5) * bb1;
  const T Rb = M01 * s.Suv + M02 * s.Suu + M12 * s.Svv + T(2) * M22 * s.Suv - bb2;
  fub = fub + (T(2) * Pb) * s.fu + Rb * s.fv;
  fvb = fvb + (T(2) * Qb) * s.fv + Rb * s.fu;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P[k].x += s.bu[k] * fub.x + s.bv[k] * fvb.x;
    P[k].y += s.bu[k] * fub.y + s.bv[k] * fvb.y;
    P[k].z += s.bu[k] * fub.z + s.bv[k] * fvb.z;
  }
  return true;
}

// ---- body collider: C = n^ . (x - a) - tau against the plane of the paired
// triangle (a, b, c), n^ the unit normal of n = (b - a) x (c - a); the body is
// kinematic (only x moves), so D = w |grad_x C|^2 + at with grad_x C = n^.
template <class T> struct BodyEval { V3<T> a, e1, e2, nh; T len, C; bool ok; };
template <class T>
__device__ __forceinline__ BodyEval<T> body_eval(V3<T> x, const T* __restrict__ bx, int4 tv, T tau) {
  BodyEval<T> e;
  e.a = {bx[3 * tv.x], bx[3 * tv.x + 1], bx[3 * tv.x + 2]};
  V3<T> b = {bx[3 * tv.y], bx[3 * tv.y + 1], bx[3 * tv.y + 2]};
  V3<T> c = {bx[3 * tv.z], bx[3 * tv.z + 1], bx[3 * tv.z + 2]};
  e.e1 = b - e.a;
  e.e2 = c - e.a;
  V3<T> n = cross(e.e1, e.e2);
  T n2 = dot(n, n);
  e.ok = n2 > T(0);
  e.len = e.ok ? sqrt(n2) : T(1);
  e.nh = (T(1) / e.len) * n;
  e.C = dot(e.nh, x - e.a) - tau;
  return e;
}

// Reverse: with r = x - a, q = (I - n^ n^T) r / |n| and q' the same for the
// adjoint gbar of grad_x C, the partials of C and of n^ . gbar give
//   bbar += e2 x Q,  cbar += Q x e1,  abar -= e2 x Q + Q x e1 + Cbar n^,
// Q = Cbar q + q'; x gets Cbar n^ (n^ does not depend on x).
template <class T>
__device__ __forceinline__ bool body_rev(Vec4<T>& P, Vec4<T> tp, const T* __restrict__ bx, int4 tv, T tau, T at,
                                         T& lbar, double* __restrict__ bgrad) {
  V3<T> x = {tp.x, tp.y, tp.z};
  BodyEval<T> ev = body_eval(x, bx, tv, tau);
  T Dn = P.w * dot(ev.nh, ev.nh) + at;
  if (!(ev.ok && ev.C < T(0) && Dn > T(0))) return false;
  T lb = tp.w;
  T dl = (-ev.C - at * lb) / Dn;
  V3<T> xb = xyz(P);
  T dlb = lbar + P.w * dot(ev.nh, xb);
  T cc = T(2) * dlb * dl / Dn;
  V3<T> gb = {P.w * (dl * xb.x - cc * ev.nh.x), P.w * (dl * xb.y - cc * ev.nh.y), P.w * (dl * xb.z - cc * ev.nh.z)};
  T Cb = -dlb / Dn;
  lbar = lbar - dlb * at / Dn;
  P.x += Cb * ev.nh.x; P.y += Cb * ev.nh.y; P.z += Cb * ev.nh.z;
  if (bgrad) {
    V3<T> r = x - ev.a;
    T il = T(1) / ev.len;
    T rn = dot(r, ev.nh), gn = dot(gb, ev.nh);
    V3<T> Q = {il * (Cb * (r.x - rn * ev.nh.x) + (gb.x - gn * ev.nh.x)),
               il * (Cb * (r.y - rn * ev.nh.y) + (gb.y - gn * ev.nh.y)),
               il * (Cb * (r.z - rn * ev.nh.z) + (gb.z - gn * ev.nh.z))};
    V3<T> db = cross(ev.e2, Q), dc = cross(Q, ev.e1);
    V3<T> da = {-(db.x + dc.x + Cb * ev.nh.x), -(db.y + dc.y + Cb * ev.nh.y), -(db.z + dc.z + Cb * ev.nh.z)};
    const int vs[3] = {tv.x, tv.y, tv.z};
    const V3<T> gs[3] = {da, db, dc};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      atomicAdd(bgrad + 3 * vs[k], (double)gs[k].x);
      atomicAdd(bgrad + 3 * vs[k] + 1, (double)gs[k].y);
      atomicAdd(bgrad + 3 * vs[k] + 2, (double)gs[k].z);
    }
  }
  return true;
}

// ===================================================================== items on global vertex state

template <class T, bool FIRST, bool TAPE>
__device__ __forceinline__ void dist_item(const Dev<T>& D, int begin, int count, int t, Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int2 e = D.d_idx[j];
  Vec4<T> a = D.X[e.x], b = D.X[e.y];
  T lb = FIRST ? T(0) : D.d_lam[j];
  bool moved;
  T ln = dist_fwd<T, TAPE>(a, b, D.d_rest[j], D.d_at[j], lb, tape + t, moved);
  D.d_lam[j] = ln;
  if (moved) { D.X[e.x] = a; D.X[e.y] = b; }
}

template <class T, bool FIRST, bool TAPE>
__device__ __forceinline__ void bend_item(const Dev<T>& D, int begin, int count, int t, Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int4 q = D.b_idx[j];
  Vec4<T> p[4] = {D.X[q.x], D.X[q.y], D.X[q.z], D.X[q.w]};
  T lb = FIRST ? T(0) : D.b_lam[j];
  bool moved;
  T ln = bend_fwd<T, TAPE>(p, D.b_th0[j], D.b_at[j], lb, tape, t, count, moved);
  D.b_lam[j] = ln;
  if (moved) { D.X[q.x] = p[0]; D.X[q.y] = p[1]; D.X[q.z] = p[2]; D.X[q.w] = p[3]; }
}

template <class T, bool FIRST, bool TAPE>
__device__ __forceinline__ void tet_item(const Dev<T>& D, int begin, int count, int t, Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  const TetRec<T>& R = D.tr;
  int4 q = R.idx[j];
  Vec4<T> p[4] = {D.X[q.x], D.X[q.y], D.X[q.z], D.X[q.w]};
  T lD = FIRST ? T(0) : D.t_lamD[j];
  T lH = FIRST ? T(0) : D.t_lamH[j];
  tet_fwd<T, TAPE>(p, load_B(R.B, R.n, j), R.atD[j], R.atH[j], R.gamma[j], lD, lH, tape + t, count);
  D.t_lamD[j] = lD;
  D.t_lamH[j] = lH;
  D.X[q.x] = p[0]; D.X[q.y] = p[1]; D.X[q.z] = p[2]; D.X[q.w] = p[3];
}

template <class T, bool FIRST, bool TAPE>
__device__ __forceinline__ void contact_item(const Dev<T>& D, int begin, int count, int t, Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int v = D.c_vid[j];
  Vec4<T> p = D.X[v];
  T lb = FIRST ? T(0) : D.c_lam[j];
  bool moved;
  T ln = contact_fwd<T, TAPE>(p, D.sph, lb, tape + t, moved);
  D.c_lam[j] = ln;
  if (moved) D.X[v] = p;
}

template <class T, bool FIRST, bool TAPE>
__device__ __forceinline__ void tri_item(const Dev<T>& D, int begin, int count, int t, Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  const TriRec<T>& R = D.mr;
  const int n = R.n;
  int4 q = R.idx[j];
  Vec4<T> p[3] = {D.X[q.x], D.X[q.y], D.X[q.z]};
  T B[4] = {R.B[j], R.B[n + j], R.B[2 * n + j], R.B[3 * n + j]};
  T at[4] = {R.at[j], R.at[n + j], R.at[2 * n + j], R.at[3 * n + j]};
  T lam[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) lam[c] = FIRST ? T(0) : D.m_lam[c * n + j];
  bool moved = tri_fwd<T, TAPE>(p, B, at, lam, tape, t, count);
#pragma unroll
  for (int c = 0; c < 3; ++c) D.m_lam[c * n + j] = lam[c];
  if (moved) { D.X[q.x] = p[0]; D.X[q.y] = p[1]; D.X[q.z] = p[2]; }
}

// one body-contact projection of vertex p against the plane of its paired
// body triangle (tri < 0: none this substep); returns lambda after it
template <class T, bool TAPE>
__device__ __forceinline__ T body_fwd(Vec4<T>& p, T lb, int tri, const Dev<T>& D, Vec4<T>* tape, bool& moved) {
  if (TAPE) *tape = Vec4<T>{p.x, p.y, p.z, lb};
  T ln = lb;
  moved = false;
  if (tri >= 0) {
    BodyEval<T> ev = body_eval(xyz(p), D.bx, D.btri[tri], D.bc_tau);
    T Dn = p.w * dot(ev.nh, ev.nh) + D.bc_at;
    if (ev.ok && ev.C < T(0) && Dn > T(0)) {
      T dl = (-ev.C - D.bc_at * lb) / Dn;
      T s = p.w * dl;
      p.x += s * ev.nh.x; p.y += s * ev.nh.y; p.z += s * ev.nh.z;
      ln = lb + dl;
      moved = true;
    }
  }
  return ln;
}

template <class T, bool FIRST, bool TAPE>
__device__ __forceinline__ void body_item(const Dev<T>& D, int begin, int count, int t, Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int v = D.bc_vid[j];
  Vec4<T> p = D.X[v];
  T lb = FIRST ? T(0) : D.bc_lam[j];
  bool moved = false;
  T ln = body_fwd<T, TAPE>(p, lb, D.bpair[j], D, tape + t, moved);
  if (moved) D.X[v] = p;
  D.bc_lam[j] = ln;
}

template <class T, bool FIRST, bool LAST>
__device__ __forceinline__ void dist_rev_item(const Dev<T>& D, int begin, int count, int t,
                                              const Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int2 e = D.d_idx[j];
  T lbar = FIRST ? T(0) : D.d_lamb[j];
  T ab = FIRST ? T(0) : D.d_ab[j];
  Vec4<T> A = D.XB[e.x], Bv = D.XB[e.y];
  if (dist_rev(A, Bv, tape[t], D.d_rest[j], D.d_at[j], lbar, ab)) { D.XB[e.x] = A; D.XB[e.y] = Bv; }
  if (LAST) D.d_acc[j] += (double)ab;
  else { D.d_lamb[j] = lbar; D.d_ab[j] = ab; }
}

template <class T, bool FIRST, bool LAST>
__device__ __forceinline__ void bend_rev_item(const Dev<T>& D, int begin, int count, int t,
                                              const Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int4 q = D.b_idx[j];
  T lbar = FIRST ? T(0) : D.b_lamb[j];
  T ab = FIRST ? T(0) : D.b_ab[j];
  Vec4<T> P[4] = {D.XB[q.x], D.XB[q.y], D.XB[q.z], D.XB[q.w]};
  if (bend_rev(P, tape, t, count, D.b_th0[j], D.b_at[j], lbar, ab)) {
    D.XB[q.x] = P[0]; D.XB[q.y] = P[1]; D.XB[q.z] = P[2]; D.XB[q.w] = P[3];
  }
  if (LAST) D.b_acc[j] += (double)ab;
  else { D.b_lamb[j] = lbar; D.b_ab[j] = ab; }
}

template <class T, bool FIRST, bool LAST>
__device__ __forceinline__ void tet_rev_item(const Dev<T>& D, int begin, int count, int t,
                                             const Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  const TetRec<T>& R = D.tr;
  int4 q = R.idx[j];
  T lbD = FIRST ? T(0) : D.t_lambD[j];
  T lbH = FIRST ? T(0) : D.t_lambH[j];
  const int nt = R.n;
  T ebD = FIRST ? T(0) : D.t_eb[j], ebH = FIRST ? T(0) : D.t_eb[nt + j], gb = FIRST ? T(0) : D.t_eb[2 * nt + j];
  Vec4<T> P[4] = {D.XB[q.x], D.XB[q.y], D.XB[q.z], D.XB[q.w]};
  if (tet_rev(P, tape + t, count, load_B(R.B, R.n, j), R.atD[j], R.atH[j], R.gamma[j], lbD, lbH, ebD, ebH, gb)) {
    D.XB[q.x] = P[0]; D.XB[q.y] = P[1]; D.XB[q.z] = P[2]; D.XB[q.w] = P[3];
  }
  if (LAST) {
    D.t_acc[j] += (double)ebD;
    D.t_acc[nt + j] += (double)ebH;
    D.t_acc[2 * nt + j] += (double)gb;
  } else {
    D.t_lambD[j] = lbD; D.t_lambH[j] = lbH;
    D.t_eb[j] = ebD; D.t_eb[nt + j] = ebH; D.t_eb[2 * nt + j] = gb;
  }
}

template <class T, bool FIRST, bool LAST>
__device__ __forceinline__ void tri_rev_item(const Dev<T>& D, int begin, int count, int t,
                                             const Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  const TriRec<T>& R = D.mr;
  const int n = R.n;
  int4 q = R.idx[j];
  T B[4] = {R.B[j], R.B[n + j], R.B[2 * n + j], R.B[3 * n + j]};
  T at[4] = {R.at[j], R.at[n + j], R.at[2 * n + j], R.at[3 * n + j]};
  T lbar[3], ab[4];
#pragma unroll
  for (int c = 0; c < 3; ++c) lbar[c] = FIRST ? T(0) : D.m_lamb[c * n + j];
#pragma unroll
  for (int c = 0; c < 4; ++c) ab[c] = FIRST ? T(0) : D.m_ab[c * n + j];
  Vec4<T> P[3] = {D.XB[q.x], D.XB[q.y], D.XB[q.z]};
  if (tri_rev(P, tape, t, count, B, at, lbar, ab)) { D.XB[q.x] = P[0]; D.XB[q.y] = P[1]; D.XB[q.z] = P[2]; }
  if (LAST) {
#pragma unroll
    for (int c = 0; c < 4; ++c) D.m_acc[c * n + j] += (double)ab[c];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) D.m_lamb[c * n + j] = lbar[c];
#pragma unroll
    for (int c = 0; c < 4; ++c) D.m_ab[c * n + j] = ab[c];
  }
}

template <class T, bool FIRST, bool LAST>
__device__ __forceinline__ void body_rev_item(const Dev<T>& D, int begin, int count, int t,
                                              const Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  const int tri = D.bpair[j];
  T lbar = FIRST ? T(0) : D.bc_lamb[j];
  if (tri >= 0) {
    int v = D.bc_vid[j];
    Vec4<T> P = D.XB[v];
    if (body_rev(P, tape[t], D.bx, D.btri[tri], D.bc_tau, D.bc_at, lbar, D.bgrad)) D.XB[v] = P;
  }
  if (!LAST) D.bc_lamb[j] = lbar;
}

template <class T, bool FIRST, bool LAST>
__device__ __forceinline__ void contact_rev_item(const Dev<T>& D, int begin, int count, int t,
                                                 const Vec4<T>* __restrict__ tape) {
  int j = begin + t;
  int v = D.c_vid[j];
  T lbar = FIRST ? T(0) : D.c_lamb[j];
  Vec4<T> sa = FIRST ? Vec4<T>{T(0), T(0), T(0), T(0)} : D.c_sacc[j];
  Vec4<T> P = D.XB[v];
  if (contact_rev(P, tape[t], D.sph, lbar, sa)) D.XB[v] = P;
  if (!LAST) D.c_lamb[j] = lbar;
  D.c_sacc[j] = sa;
}

// ===================================================================== per-vertex items

// substep start: x_prev = x; v += h (g + w f) for free vertices; x += h v
template <class T> __device__ __forceinline__ void predict_item(const Dev<T>& D, int k, const T* __restrict__ f) {
  Vec4<T> x = D.X[k], v = D.Vv[k];
  D.Xp[k] = x;
  if (x.w > T(0)) {
    T fx = T(0), fy = T(0), fz = T(0);
    if (f) { fx = f[3 * k]; fy = f[3 * k + 1]; fz = f[3 * k + 2]; }
    v.x += D.h * (D.gx + x.w * fx);
    v.y += D.h * (D.gy + x.w * fy);
    v.z += D.h * (D.gz + x.w * fz);
    D.Vv[k] = v;
  }
  x.x += D.h * v.x; x.y += D.h * v.y; x.z += D.h * v.z;
  D.X[k] = x;
}
// substep end: v = (x - x_prev) / h
template <class T> __device__ __forceinline__ void velocity_item(const Dev<T>& D, int k) {
  Vec4<T> x = D.X[k], xp = D.Xp[k];
  D.Vv[k] = Vec4<T>{(x.x - xp.x) * D.inv_h, (x.y - xp.y) * D.inv_h, (x.z - xp.z) * D.inv_h, T(0)};
}
// reverse of v = (x - x_prev)/h, first half: xbar += vbar / h
template <class T> __device__ __forceinline__ void rev_velocity_item(const Dev<T>& D, int k) {
  Vec4<T> p = D.XB[k], v = D.VB[k];
  p.x += v.x * D.inv_h; p.y += v.y * D.inv_h; p.z += v.z * D.inv_h;
  D.XB[k] = p;
}
// reverse of the prediction plus the x_prev half of the velocity update:
//   vbar_mid = h xbar (free), fbar += h w vbar_mid, xbar = xbar - vbar_old / h,
//   vbar = vbar_mid
template <class T> __device__ __forceinline__ void rev_predict_item(const Dev<T>& D, int k, T* __restrict__ fbar) {
  Vec4<T> p = D.XB[k], v = D.VB[k];
  Vec4<T> vm = {T(0), T(0), T(0), T(0)};
  if (p.w > T(0)) { vm.x = D.h * p.x; vm.y = D.h * p.y; vm.z = D.h * p.z; }
  if (fbar) {
    T s = D.h * p.w;
    fbar[3 * k] += s * vm.x; fbar[3 * k + 1] += s * vm.y; fbar[3 * k + 2] += s * vm.z;
  }
  p.x -= v.x * D.inv_h; p.y -= v.y * D.inv_h; p.z -= v.z * D.inv_h;
  D.XB[k] = p;
  D.VB[k] = vm;
}

// ===================================================================== plain kernels (one launch per set)

__device__ __forceinline__ int thread_item(int count) {
  int t = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x + threadIdx.x;
  return t < count ? t : -1;
}

// The per-set kernels read the parameter block from device memory (stored
// once per substep by k_store_dev): a launch then carries a pointer and three
// words of arguments instead of the whole block, which matters where the
// step is a long chain of short dependent launches.
#define XPBD_SET_KERNEL(NAME, ITEM, TAPE_T)                                                              \
  template <class T, bool F1, bool F2>                                                                   \
  __global__ __launch_bounds__(kMaxBlock) void NAME(const Dev<T>* __restrict__ Dp, int begin, int count, \
                                                    TAPE_T* tape) {                                      \
    int t = thread_item(count);                                                                          \
    if (t >= 0) ITEM<T, F1, F2>(*Dp, begin, count, t, tape);                                             \
  }
XPBD_SET_KERNEL(k_dist, dist_item, Vec4<T>)
XPBD_SET_KERNEL(k_bend, bend_item, Vec4<T>)
XPBD_SET_KERNEL(k_tet, tet_item, Vec4<T>)
XPBD_SET_KERNEL(k_contact, contact_item, Vec4<T>)
XPBD_SET_KERNEL(k_tri, tri_item, Vec4<T>)
XPBD_SET_KERNEL(k_body, body_item, Vec4<T>)
XPBD_SET_KERNEL(k_dist_rev, dist_rev_item, const Vec4<T>)
XPBD_SET_KERNEL(k_bend_rev, bend_rev_item, const Vec4<T>)
XPBD_SET_KERNEL(k_tet_rev, tet_rev_item, const Vec4<T>)
XPBD_SET_KERNEL(k_contact_rev, contact_rev_item, const Vec4<T>)
XPBD_SET_KERNEL(k_tri_rev, tri_rev_item, const Vec4<T>)
XPBD_SET_KERNEL(k_body_rev, body_rev_item, const Vec4<T>)
#undef XPBD_SET_KERNEL

// one thread stores the parameter block the per-set kernels of a substep read
template <class T> __global__ __launch_bounds__(64) void k_store_dev(Dev<T> D, Dev<T>* __restrict__ out) {
  if (threadIdx.x == 0) *out = D;
}

template <class T> __global__ __launch_bounds__(kBlock) void k_predict(Dev<T> D, const T* f) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < D.V) predict_item(D, k, f);
}
template <class T> __global__ __launch_bounds__(kBlock) void k_velocity(Dev<T> D) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < D.V) velocity_item(D, k);
}
template <class T> __global__ __launch_bounds__(kBlock) void k_rev_velocity(Dev<T> D) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < D.V) rev_velocity_item(D, k);
}
template <class T> __global__ __launch_bounds__(kBlock) void k_rev_predict(Dev<T> D, T* fbar) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < D.V) rev_predict_item(D, k, fbar);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_pack(const T* __restrict__ x0, const T* __restrict__ v0,
                                                 const T* __restrict__ w, Vec4<T>* __restrict__ X,
                                                 Vec4<T>* __restrict__ Vv, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  T wk = w[k];
  X[k] = Vec4<T>{x0[3 * k], x0[3 * k + 1], x0[3 * k + 2], wk};
  if (wk > T(0)) Vv[k] = Vec4<T>{v0[3 * k], v0[3 * k + 1], v0[3 * k + 2], T(0)};
  else Vv[k] = Vec4<T>{T(0), T(0), T(0), T(0)};
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_unpack(const Vec4<T>* __restrict__ X, T* __restrict__ out, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  Vec4<T> p = X[k];
  out[3 * k] = p.x; out[3 * k + 1] = p.y; out[3 * k + 2] = p.z;
}

// adjoint state init: xbar = 0 (keeping w), vbar = dL/dv_final or 0
template <class T>
__global__ __launch_bounds__(kBlock) void k_adj_init(Vec4<T>* __restrict__ XB, Vec4<T>* __restrict__ VB,
                                                     const T* __restrict__ w, const T* __restrict__ dv, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  XB[k] = Vec4<T>{T(0), T(0), T(0), w[k]};
  if (dv) VB[k] = Vec4<T>{dv[3 * k], dv[3 * k + 1], dv[3 * k + 2], T(0)};
  else VB[k] = Vec4<T>{T(0), T(0), T(0), T(0)};
}

// xbar += dL/dx(f)
template <class T>
__global__ __launch_bounds__(kBlock) void k_adj_inject(Vec4<T>* __restrict__ XB, const T* __restrict__ g, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  Vec4<T> p = XB[k];
  p.x += g[3 * k]; p.y += g[3 * k + 1]; p.z += g[3 * k + 2];
  XB[k] = p;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ p, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// ===================================================================== parameters

__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

// at[i] = alpha[perm[i]] / h^2 (internal order);  flag |= non-finite
template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_alpha(const T* __restrict__ alpha, const int* __restrict__ perm,
                                                         T* __restrict__ at, T inv_h2, int n, int* __restrict__ flag) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T a = alpha ? alpha[perm[i]] : T(0);
  if (!finite_d((double)a) || a < T(0)) *flag = 1;
  at[i] = a * inv_h2;
}

// per tet: mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu)),
// atD = 1/(mu V h^2), atH = 1/(lambda V h^2), gamma = 1 + mu/lambda (or 1)
template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_tet(const T* __restrict__ E, const int* __restrict__ perm,
                                                       const double* __restrict__ nu, const double* __restrict__ vol,
                                                       T* __restrict__ atD, T* __restrict__ atH, T* __restrict__ gam,
                                                       double inv_h2, int gamma_one, int n, int* __restrict__ flag) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double e = (double)E[perm[i]];
  if (!finite_d(e) || !(e > 0.0)) *flag = 1;
  double v = nu[i], V = vol[i];
  double mu = e / (2.0 * (1.0 + v));
  double la = e * v / ((1.0 + v) * (1.0 - 2.0 * v));
  atD[i] = (T)(inv_h2 / (mu * V));
  atH[i] = (T)(inv_h2 / (la * V));
  gam[i] = gamma_one ? T(1) : (T)(1.0 + mu / la);
}

// gradient scatter: out[perm[i]] = acc[i] * scale     (dist, bend)
__global__ __launch_bounds__(kBlock) void k_scatter_alpha_grad(const double* __restrict__ acc, const int* __restrict__ perm,
                                                               double* __restrict__ out, double scale, int n) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  out[perm[i]] = acc[i] * scale;
}
// acc = [abar~_D alpha~_D | abar~_H alpha~_H | gammabar] per tet (internal order).
// At fixed nu both compliances scale as 1/E and gamma does not depend on E:
// dL/dE = -(acc_D + acc_H) / E
template <class T>
__global__ __launch_bounds__(kBlock) void k_scatter_E_grad(const double* __restrict__ acc, const int* __restrict__ perm,
                                                           const T* __restrict__ E, double* __restrict__ out, int n) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int u = perm[i];
  out[u] = -(acc[i] + acc[n + i]) / (double)E[u];
}
// Lame parameters (Sec. 5.2): alpha_D = 1/(mu V), alpha_H = 1/(lambda V),
// gamma = 1 + mu/lambda (1 with gamma_one):
// dL/dmu = -acc_D / mu + gammabar / lambda,
// dL/dlambda = -acc_H / lambda - gammabar mu / lambda^2
template <class T>
__global__ __launch_bounds__(kBlock) void k_scatter_lame_grad(const double* __restrict__ acc, const int* __restrict__ perm,
                                                              const T* __restrict__ mu, const T* __restrict__ la,
                                                              double* __restrict__ out_mu, double* __restrict__ out_la,
                                                              int gamma_one, int n) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int u = perm[i];
  double m = (double)mu[u], l = (double)la[u], g = gamma_one ? 0.0 : acc[2 * n + i];
  if (out_mu) out_mu[u] = -acc[i] / m + g / l;
  if (out_la) out_la[u] = -acc[n + i] / l - g * m / (l * l);
}
// Membrane compliance per triangle from its coefficients (C00, C01, C11, C22)
// (caller order, [n][4]): alpha = (A K)^-1 with K = [[C00, C01, 0],
// [C01, C11, 0], [0, 0, C22]]; at = alpha / h^2 keeps the 2x2 block and the
// shear entry.  flag |= non-finite or K not positive definite.
template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_tri(const T* __restrict__ coef, const int* __restrict__ perm,
                                                       const double* __restrict__ area, T* __restrict__ at,
                                                       double inv_h2, int n, int* __restrict__ flag) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const T* q = coef + 4 * (size_t)perm[i];
  double c00 = (double)q[0], c01 = (double)q[1], c11 = (double)q[2], c22 = (double)q[3];
  double det = c00 * c11 - c01 * c01;
  if (!finite_d(c00) || !finite_d(c01) || !finite_d(c11) || !finite_d(c22) || !(c00 > 0.0) || !(c22 > 0.0) ||
      !(det > 0.0))
    *flag = 1;
  double s = inv_h2 / area[i];
  at[i] = (T)(s * c11 / det);
  at[n + i] = (T)(-s * c01 / det);
  at[2 * n + i] = (T)(s * c00 / det);
  at[3 * n + i] = (T)(s / c22);
}
// dL/dK = -A h^2 at Sym(atbar) at with at = K^-1 / (A h^2), i.e.
// -K^-1 Sym(atbar) K^-1 / (A h^2); acc = Sym(atbar) entries (00, 01 + 10,
// 11, 22); C01 enters K twice.
template <class T>
__global__ __launch_bounds__(kBlock) void k_scatter_tri_grad(const double* __restrict__ acc, const int* __restrict__ perm,
                                                             const T* __restrict__ coef, const double* __restrict__ area,
                                                             double* __restrict__ out, double inv_h2, int n) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int u = perm[i];
  const T* q = coef + 4 * (size_t)u;
  double c00 = (double)q[0], c01 = (double)q[1], c11 = (double)q[2], c22 = (double)q[3];
  double det = c00 * c11 - c01 * c01;
  double i00 = c11 / det, i01 = -c01 / det, i11 = c00 / det, i22 = 1.0 / c22;   // K^-1
  double s00 = acc[i], s01 = 0.5 * acc[n + i], s11 = acc[2 * n + i], s22 = acc[3 * n + i];
  // Y = K^-1 S K^-1 on the 2x2 block
  double a00 = i00 * s00 + i01 * s01, a01 = i00 * s01 + i01 * s11;
  double a10 = i01 * s00 + i11 * s01, a11 = i01 * s01 + i11 * s11;
  double y00 = a00 * i00 + a01 * i01, y01 = a00 * i01 + a01 * i11, y11 = a10 * i01 + a11 * i11;
  double k = -inv_h2 / area[i];
  double* o = out + 4 * (size_t)u;
  o[0] = k * y00;
  o[1] = 2.0 * k * y01;
  o[2] = k * y11;
  o[3] = k * i22 * s22 * i22;
}

// Body pairing: a uniform grid over the body's bounding box grown by the
// search radius r, each cell listing (ascending) the triangles whose own box
// grown by r meets it, so every triangle within r of a point is listed in the
// point's cell.
struct BodyGrid {
  double lo[3];
  double inv_cell;
  int dims[3];
  const int* off;    // [cells + 1]
  const int* tris;   // cell lists
};

// squared distance from p to triangle (a, b, c): the closest point found by
// classifying p against the triangle's Voronoi regions (vertex, edge or face)
// with barycentric dot products, Ericson, Real-Time Collision Detection
// (2005), Sec. 5.1.5
__device__ __forceinline__ double point_tri_d2(V3<double> p, V3<double> a, V3<double> b, V3<double> c) {
  V3<double> ab = b - a, ac = c - a, ap = p - a;
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  V3<double> q;
  if (d1 <= 0.0 && d2 <= 0.0) { q = a; }
  else {
    V3<double> bp = p - b;
    double d3 = dot(ab, bp), d4 = dot(ac, bp);
    double vc = d1 * d4 - d3 * d2;
    if (d3 >= 0.0 && d4 <= d3) { q = b; }
    else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) { double t = d1 / (d1 - d3); q = a + t * ab; }
    else {
      V3<double> cp = p - c;
      double d5 = dot(ab, cp), d6 = dot(ac, cp);
      double vb = d5 * d2 - d1 * d6;
      double va = d3 * d6 - d5 * d4;
      if (d6 >= 0.0 && d5 <= d6) { q = c; }
      else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) { double t = d2 / (d2 - d6); q = a + t * ac; }
      else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        q = b + t * (c - b);
      } else {
        double den = 1.0 / (va + vb + vc);
        q = a + (vb * den) * ab + (vc * den) * ac;
      }
    }
  }
  V3<double> r = p - q;
  return dot(r, r);
}

// pair each body-contact item with its closest triangle within r, -1 if
// none: the least distance d2min over the cell's triangles, then the
// lowest-index triangle with d2 <= d2min (1 + 1e-9) + 1e-20 (a point nearest
// to an edge or corner shared by several triangles is equally near to each;
// the margin makes that choice independent of how the distance rounds)
template <class T>
__global__ __launch_bounds__(kBlock) void k_body_detect(const Vec4<T>* __restrict__ X, const int* __restrict__ vid, int n,
                                                        const T* __restrict__ bx, const int4* __restrict__ btri,
                                                        BodyGrid G, double r2, int* __restrict__ pair) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  Vec4<T> xp = X[vid[j]];
  V3<double> p = {(double)xp.x, (double)xp.y, (double)xp.z};
  int ci[3];
  const double pc[3] = {p.x, p.y, p.z};
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double u = (pc[a] - G.lo[a]) * G.inv_cell;
    inside = inside && u >= 0.0 && u < (double)G.dims[a];
    ci[a] = inside ? (int)u : 0;
  }
  int best = -1;
  if (inside) {
    const int cell = (ci[0] * G.dims[1] + ci[1]) * G.dims[2] + ci[2];
    auto d2_of = [&](int t) {
      int4 tv = btri[t];
      V3<double> a = {(double)bx[3 * tv.x], (double)bx[3 * tv.x + 1], (double)bx[3 * tv.x + 2]};
      V3<double> b = {(double)bx[3 * tv.y], (double)bx[3 * tv.y + 1], (double)bx[3 * tv.y + 2]};
      V3<double> c = {(double)bx[3 * tv.z], (double)bx[3 * tv.z + 1], (double)bx[3 * tv.z + 2]};
      return point_tri_d2(p, a, b, c);
    };
    double bd = INFINITY;
    for (int q = G.off[cell]; q < G.off[cell + 1]; ++q) bd = fmin(bd, d2_of(G.tris[q]));
    if (bd <= r2) {
      const double lim = bd * (1.0 + 1e-9) + 1e-20;
      for (int q = G.off[cell]; q < G.off[cell + 1]; ++q) {
        int t = G.tris[q];
        if ((best < 0 || t < best) && d2_of(t) <= lim) best = t;
      }
    }
  }
  pair[j] = best;
}

// Material clusters: the gradient of material m is the sum of the per-tet
// terms above over its tets items[off[m] .. off[m+1]) (internal indices in
// ascending order), one workgroup per material with strided partial sums and
// a fixed tree, so the sum does not depend on timing.  E != nullptr: Young's
// moduli (into oE); else Lame parameters (into oMu, oLa, either may be null).
template <class T>
__global__ __launch_bounds__(kBlock) void k_material_grad(const double* __restrict__ acc, const int* __restrict__ off,
                                                          const int* __restrict__ items, const T* __restrict__ E,
                                                          const T* __restrict__ mu, const T* __restrict__ la,
                                                          double* __restrict__ oE, double* __restrict__ oMu,
                                                          double* __restrict__ oLa, int gamma_one, int n) {
  __shared__ double s0[kBlock], s1[kBlock];
  const int m = blockIdx.x;
  const int beg = off[m], end = off[m + 1];
  double a = 0.0, b = 0.0;
  if (E) {
    const double e = (double)E[m];
    for (int q = beg + (int)threadIdx.x; q < end; q += kBlock) {
      int j = items[q];
      a += -(acc[j] + acc[n + j]) / e;
    }
  } else {
    const double mm = (double)mu[m], l = (double)la[m];
    for (int q = beg + (int)threadIdx.x; q < end; q += kBlock) {
      int j = items[q];
      double g = gamma_one ? 0.0 : acc[2 * n + j];
      a += -acc[j] / mm + g / l;
      b += -acc[n + j] / l - g * mm / (l * l);
    }
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (E) oE[m] = s0[0];
    if (oMu) oMu[m] = s0[0];
    if (oLa) oLa[m] = s1[0];
  }
}

// per tet from Lame parameters: atD = 1/(mu V h^2), atH = 1/(lambda V h^2),
// gamma = 1 + mu/lambda (or 1); flag |= non-positive or non-finite
template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_tet_lame(const T* __restrict__ mu, const T* __restrict__ la,
                                                            const int* __restrict__ perm, const double* __restrict__ vol,
                                                            T* __restrict__ atD, T* __restrict__ atH, T* __restrict__ gam,
                                                            double inv_h2, int gamma_one, int n, int* __restrict__ flag) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int u = perm[i];
  double m = (double)mu[u], l = (double)la[u], V = vol[i];
  if (!finite_d(m) || !finite_d(l) || !(m > 0.0) || !(l > 0.0)) *flag = 1;
  atD[i] = (T)(inv_h2 / (m * V));
  atH[i] = (T)(inv_h2 / (l * V));
  gam[i] = gamma_one ? T(1) : (T)(1.0 + m / l);
}

// Deterministic block reduction of the per-contact sphere adjoints into the
// FP64 sphere gradient (fixed order: strided partial sums, then a tree).
// `order` lists the set's items by ascending vertex, so the sum does not
// depend on how the items are laid out.
template <class T, int NT>
__device__ __forceinline__ void sphere_reduce_block(const Vec4<T>* __restrict__ sacc, const int* __restrict__ order,
                                                    int begin, int count, double* __restrict__ out, double (*sh)[NT]) {
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int i = threadIdx.x; i < count; i += NT) {
    Vec4<T> v = sacc[begin + order[begin + i]];
    s0 += v.x; s1 += v.y; s2 += v.z; s3 += v.w;
  }
  sh[0][threadIdx.x] = s0; sh[1][threadIdx.x] = s1; sh[2][threadIdx.x] = s2; sh[3][threadIdx.x] = s3;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4 && out) out[threadIdx.x] += sh[threadIdx.x][0];
  __syncthreads();
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_sphere_reduce(const Vec4<T>* __restrict__ sacc, const int* __restrict__ order,
                                                          int begin, int count, double* __restrict__ out) {
  __shared__ double sh[4][kBlock];
  sphere_reduce_block<T, kBlock>(sacc, order, begin, count, out, sh);
}

// FP64 goal: per-block partial sums of 1/2 |W (x - x*)|^2 on masked frames,
// and dL/dx = W^2 (x - x*) (0 on unmasked frames); W = I or diag(w) with
// one weight per vertex (x is [V][3], element i belongs to vertex i / 3)
template <class T>
__global__ __launch_bounds__(kBlock) void k_goal(const T* __restrict__ x, const T* __restrict__ tg,
                                                 const double* __restrict__ w, T* __restrict__ g, size_t n, int on,
                                                 double* __restrict__ part) {
  __shared__ double sh[kBlock];
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    double d = on ? (double)x[i] - (double)tg[i] : 0.0;
    if (w) {
      double ww = w[i / 3] * w[i / 3];
      if (g) g[i] = on ? (T)(ww * d) : T(0);
      s = 0.5 * ww * d * d;
    } else {
      if (g) g[i] = on ? (T)(x[i] - tg[i]) : T(0);
      s = 0.5 * d * d;
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ __launch_bounds__(1024) void k_sum_parts(const double* __restrict__ part, size_t n, double* __restrict__ out,
                                                    int accumulate) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 1024) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = accumulate ? *out + sh[0] : sh[0];
}

// ===================================================================== LDS group kernels
// A group is a run of consecutive independent sets together with a vertex
// partition under which every constraint of those sets has all its vertices
// in one patch.  One workgroup per patch stages the patch's vertices and the
// records of its constraints in LDS, runs the group's sets in schedule order
// with a workgroup barrier between sets, and writes back.  Patches share no
// vertex inside the group, so the result equals running the sets one launch
// at a time, bit for bit.
//
// The constraints of a group live in global memory as patch-major images
// laid out exactly like the LDS copy (set after set, each padded to 32
// bytes), so staging is one contiguous 16-byte copy per patch.  Each
// constraint has a constant entry (vertex slots in the patch's tile, rest
// data, compliances), shared by the forward and the reverse, and mutable
// state in two separate images of the same layout: the multipliers of the
// forward and the reverse's multiplier and compliance adjoints, stored per
// set as arrays of the set's items.  A launch reads the constant image and
// writes back only the state it changes.  The forward writes the adjoint's
// record of projection inputs in the same patch-major layout, which the
// reverse stages the same way.

constexpr int kMaxGroupSets = 64;

template <class T> struct SDist { T rest, at; unsigned l; };
template <class T> struct SBend { T th0, at; unsigned l01, l23; };
template <class T> struct STet { T B[9]; T atD, atH, gam; unsigned l01, l23; };
template <class T> struct SCon { unsigned l; };
template <class T> struct STri { T B[4]; T at[4]; unsigned l01, l2; };   // Dm^-1, at00 at01 at11 at22
template <class T> struct SBody { unsigned l; int j; };   // vertex slot, item (its substep pairing)

__host__ __device__ __forceinline__ size_t al32(size_t b) { return (b + 31) & ~(size_t)31; }
__device__ __forceinline__ int lo16(unsigned v) { return (int)(v & 0xffffu); }
__device__ __forceinline__ int hi16(unsigned v) { return (int)(v >> 16); }

template <class T> __host__ __device__ inline size_t rec_bytes(int type) {
  return type == 0 ? sizeof(SDist<T>) : type == 1 ? sizeof(SBend<T>) : type == 2 ? sizeof(STet<T>)
         : type == 4 ? sizeof(STri<T>) : type == 5 ? sizeof(SBody<T>) : sizeof(SCon<T>);
}
// words of mutable state per item, each word an array over the set's items:
// forward lambda (tets lambda_D, lambda_H); reverse lambda_bar and the
// compliance adjoint (tets lambda_bar_D, lambda_bar_H, the two compliance
// adjoints and gamma_bar; contacts the sphere adjoint, a Vec4 array, then
// lambda_bar; membranes three multipliers, then their three adjoints and
// the four compliance adjoints; body contacts lambda, then lambda_bar)
__host__ __device__ inline size_t fmul_words(int type) { return type == 2 ? 2 : type == 4 ? 3 : 1; }
__host__ __device__ inline size_t rmul_words(int type) { return type <= 1 ? 2 : type == 4 ? 7 : type == 5 ? 1 : 5; }
__host__ __device__ inline size_t tape_words(int type) { return type == 1 ? 10 : type == 2 || type == 4 ? 12 : 4; }

struct GroupDev {
  const int* pv_start;      // [P + 1] patch vertex ranges
  const int* pv;            // global vertex of each patch slot
  const int* cnt;           // [P][nset] items of each set in each patch
  const int* set_type;      // [nset]
  const long long* img;     // [P] byte offset of each patch's constant entries
  const long long* fmul;    // [P] ... forward multipliers
  const long long* rmul;    // [P] ... reverse state
  const long long* tpos;    // [P] byte offset of each patch's record of inputs in the group's chunk
  const int* rec_first;     // [P][nset] internal index of the patch's first item in each set
  int nset, P;
  long long tape_off;       // byte offset of the group's chunk inside one iteration's record
  // snapshot records: offsets of the group's staged positions and of its
  // multipliers inside one iteration's snapshot, and the byte offset of the
  // group's first patch in the forward state image
  long long snap_x_off, snap_l_off, fmul_lo;
};

// Workgroup barrier that orders LDS only: the group kernels share nothing
// through global memory between threads (a replayed record in global scratch
// is read back only by the thread that wrote it), so outstanding global
// stores (records of projection inputs, snapshots) keep draining across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void copy16(void* dst, const void* src, size_t bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

// A group launch stages its patch's item count and the type of every set
// (at most kMaxGroupSets) in LDS first, since global loads of them at each set
// step would put a memory round trip ahead of the set's own loads.
__device__ __forceinline__ void stage_sets(const GroupDev& G, int p, int* s_cnt, int* s_ty) {
  for (int q = threadIdx.x; q < G.nset; q += blockDim.x) {
    s_cnt[q] = G.cnt[(size_t)p * G.nset + q];
    s_ty[q] = G.set_type[q];
  }
  lds_barrier();
}

// The group's sets of one iteration in schedule order on the vertex tile sX
// (LDS), one thread per item with a workgroup barrier between sets: constant
// entries from r, multipliers from m (written back when KEEP), the record of
// each projection's inputs to gt when TAPE.  The forward launch and the
// reverse's replay of a launch (records kept as snapshots) both run this, so
// they compute every projection bit for bit alike.
template <class T, bool FIRST, bool TAPE, bool HEAVY, bool KEEP>
__device__ __forceinline__ void group_sets_fwd(const Dev<T>& D, const GroupDev& G, const int* cnt, const int* sty,
                                               Vec4<T>* sX, const unsigned char* r, unsigned char* m, char* gt) {
  const int tid = threadIdx.x, kB = blockDim.x;
  for (int q = 0; q < G.nset; ++q) {
    const int n = cnt[q], ty = sty[q];
    Vec4<T>* tape = reinterpret_cast<Vec4<T>*>(gt);
    T* lam = reinterpret_cast<T*>(m);
    switch (ty) {
      case 0:
        for (int i = tid; i < n; i += kB) {
          const SDist<T> s = reinterpret_cast<const SDist<T>*>(r)[i];
          int la = lo16(s.l), lb = hi16(s.l);
          Vec4<T> a = sX[la], bb = sX[lb];
          T l0 = FIRST ? T(0) : lam[i];
          bool moved;
          T ln = dist_fwd<T, TAPE>(a, bb, s.rest, s.at, l0, tape + i, moved);
          if (moved) { sX[la] = a; sX[lb] = bb; }
          if (KEEP) lam[i] = ln;
        }
        break;
      case 1:
        for (int i = tid; i < n; i += kB) {
          const SBend<T> s = reinterpret_cast<const SBend<T>*>(r)[i];
          int l[4] = {lo16(s.l01), hi16(s.l01), lo16(s.l23), hi16(s.l23)};
          Vec4<T> pp[4] = {sX[l[0]], sX[l[1]], sX[l[2]], sX[l[3]]};
          T l0 = FIRST ? T(0) : lam[i];
          bool moved;
          T ln = bend_fwd<T, TAPE>(pp, s.th0, s.at, l0, tape, i, n, moved);
          if (moved) { sX[l[0]] = pp[0]; sX[l[1]] = pp[1]; sX[l[2]] = pp[2]; sX[l[3]] = pp[3]; }
          if (KEEP) lam[i] = ln;
        }
        break;
      case 2:
        if constexpr (HEAVY)
        for (int i = tid; i < n; i += kB) {
          const STet<T>& s = reinterpret_cast<const STet<T>*>(r)[i];
          int l[4] = {lo16(s.l01), hi16(s.l01), lo16(s.l23), hi16(s.l23)};
          Vec4<T> pp[4] = {sX[l[0]], sX[l[1]], sX[l[2]], sX[l[3]]};
          M3<T> B;
#pragma unroll
          for (int k = 0; k < 9; ++k) B.m[k / 3][k % 3] = s.B[k];
          T lD = FIRST ? T(0) : lam[i], lH = FIRST ? T(0) : lam[n + i];
          tet_fwd<T, TAPE>(pp, B, s.atD, s.atH, s.gam, lD, lH, tape + i, n);
          if (KEEP) { lam[i] = lD; lam[n + i] = lH; }
          sX[l[0]] = pp[0]; sX[l[1]] = pp[1]; sX[l[2]] = pp[2]; sX[l[3]] = pp[3];
        }
        break;
      case 4:
        if constexpr (HEAVY)
        for (int i = tid; i < n; i += kB) {
          const STri<T>& s = reinterpret_cast<const STri<T>*>(r)[i];
          int l[3] = {lo16(s.l01), hi16(s.l01), (int)s.l2};
          Vec4<T> pp[3] = {sX[l[0]], sX[l[1]], sX[l[2]]};
          T B[4] = {s.B[0], s.B[1], s.B[2], s.B[3]}, at[4] = {s.at[0], s.at[1], s.at[2], s.at[3]};
          T lm[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) lm[c] = FIRST ? T(0) : lam[c * n + i];
          bool moved = tri_fwd<T, TAPE>(pp, B, at, lm, tape, i, n);
#pragma unroll
          for (int c = 0; c < 3; ++c) if (KEEP) lam[c * n + i] = lm[c];
          if (moved) { sX[l[0]] = pp[0]; sX[l[1]] = pp[1]; sX[l[2]] = pp[2]; }
        }
        break;
      case 5:
        if constexpr (HEAVY)
        for (int i = tid; i < n; i += kB) {
          const SBody<T> e = reinterpret_cast<const SBody<T>*>(r)[i];
          Vec4<T> pp = sX[e.l];
          T l0 = FIRST ? T(0) : lam[i];
          bool moved = false;
          T ln = body_fwd<T, TAPE>(pp, l0, D.bpair[e.j], D, tape + i, moved);
          if (moved) sX[e.l] = pp;
          if (KEEP) lam[i] = ln;
        }
        break;
      default:
        for (int i = tid; i < n; i += kB) {
          const int l = (int)reinterpret_cast<const SCon<T>*>(r)[i].l;
          Vec4<T> pp = sX[l];
          T l0 = FIRST ? T(0) : lam[i];
          bool moved;
          T ln = contact_fwd<T, TAPE>(pp, D.sph, l0, tape + i, moved);
          if (moved) sX[l] = pp;
          if (KEEP) lam[i] = ln;
        }
        break;
    }
    r += al32((size_t)n * rec_bytes<T>(ty));
    m += al32((size_t)n * fmul_words(ty) * sizeof(T));
    if (TAPE) gt += al32((size_t)n * tape_words(ty) * sizeof(T));
    lds_barrier();
  }
}

// RL: the patch's constant entries and state are staged in LDS with its
// vertices (one bulk copy in, the state copied out); otherwise only the
// vertex tile is in LDS and each set's entries are read, and its state read
// and written, in place in the global images, which keeps the workgroup's
// LDS small so many patches run per CU.  HEAVY: the group has tet or
// membrane sets; the kernels without those projections need far fewer
// registers, so more waves of a distance / bending group run per SIMD.
// REC: 0 no record; 1 the record of every projection's inputs (patch-major,
// at tape_iter + G.tape_off + G.tpos[p]); 2 a snapshot of the launch's
// inputs instead: the patch's vertex positions (3 words per staged vertex at
// tape_iter + G.snap_x_off) and, after the first iteration, its multipliers
// (the forward state image of the patch, at tape_iter + G.snap_l_off), from
// which the reverse replays the launch.
template <class T, bool FIRST, int REC, bool RL, bool HEAVY>
__global__ __launch_bounds__(kBlock) void k_group_fwd(Dev<T> D, GroupDev G, const char* __restrict__ img,
                                                      char* __restrict__ fmul, char* __restrict__ tape_iter) {
  extern __shared__ __align__(32) unsigned char smem[];
  __shared__ int cnt[kMaxGroupSets], sty[kMaxGroupSets];
  const int p = blockIdx.x, tid = threadIdx.x, kB = blockDim.x;
  const int v0 = G.pv_start[p], nv = G.pv_start[p + 1] - v0;
  stage_sets(G, p, cnt, sty);
  Vec4<T>* sX = reinterpret_cast<Vec4<T>*>(smem);
  const char* gimg = img + G.img[p];
  char* gmul = fmul + G.fmul[p];
  unsigned char* lrec = smem + al32((size_t)nv * sizeof(Vec4<T>));
  size_t rbytes = 0, mbytes = 0;
  if (RL || REC == 2)
    for (int q = 0; q < G.nset; ++q) {
      rbytes += al32((size_t)cnt[q] * rec_bytes<T>(sty[q]));
      mbytes += al32((size_t)cnt[q] * fmul_words(sty[q]) * sizeof(T));
    }
  const unsigned char* r = RL ? lrec : reinterpret_cast<const unsigned char*>(gimg);
  unsigned char* m = RL ? lrec + rbytes : reinterpret_cast<unsigned char*>(gmul);
  T* snx = REC == 2 ? reinterpret_cast<T*>(tape_iter + G.snap_x_off) + 3 * (size_t)v0 : nullptr;
  for (int i = tid; i < nv; i += kB) {
    const Vec4<T> x = D.X[G.pv[v0 + i]];
    sX[i] = x;
    if (REC == 2) { snx[3 * i] = x.x; snx[3 * i + 1] = x.y; snx[3 * i + 2] = x.z; }
  }
  if (RL) {
    copy16(lrec, gimg, rbytes);
    if (!FIRST) copy16(lrec + rbytes, gmul, mbytes);   // the first iteration starts from lambda = 0
  }
  // the multipliers as this launch finds them (each thread's copy has its
  // loads back before the barrier below, ahead of any update in place)
  if (REC == 2 && !FIRST) copy16(tape_iter + G.snap_l_off + (G.fmul[p] - G.fmul_lo), gmul, mbytes);
  lds_barrier();
  char* gt = REC == 1 ? tape_iter + G.tape_off + G.tpos[p] : nullptr;
  group_sets_fwd<T, FIRST, REC == 1, HEAVY, true>(D, G, cnt, sty, sX, r, m, gt);
  for (int i = tid; i < nv; i += kB) D.X[G.pv[v0 + i]] = sX[i];
  if (RL) copy16(gmul, lrec + rbytes, mbytes);
}

// The reverse of one set of a group launch (the adjoint of its projections in
// reverse item order does not matter: the items of a set share no vertex):
// constant entries from r, the reverse state read and written in place at m,
// the record of the forward's inputs from t, the vertex adjoints in the LDS
// tile sX.  AB: the distance and bending compliance adjoints are
// accumulated (their words of the reverse state read and written); without
// it they are neither read, written nor computed.
template <class T, bool FIRST, bool HEAVY, bool AB>
__device__ __forceinline__ void group_set_rev(const Dev<T>& D, int ty, int n, const unsigned char* r,
                                              unsigned char* m, const unsigned char* t, Vec4<T>* sX) {
  const int tid = threadIdx.x, kB = blockDim.x;
  const Vec4<T>* st = reinterpret_cast<const Vec4<T>*>(t);
  T* mb = reinterpret_cast<T*>(m);
  switch (ty) {
    case 0:
      for (int i = tid; i < n; i += kB) {
        const SDist<T> s = reinterpret_cast<const SDist<T>*>(r)[i];
        int la = lo16(s.l), lb = hi16(s.l);
        Vec4<T> A = sX[la], Bv = sX[lb];
        T lbar = FIRST ? T(0) : mb[i], ab = FIRST || !AB ? T(0) : mb[n + i];
        if (dist_rev(A, Bv, st[i], s.rest, s.at, lbar, ab)) { sX[la] = A; sX[lb] = Bv; }
        mb[i] = lbar;
        if (AB) mb[n + i] = ab;
      }
      break;
    case 1:
      for (int i = tid; i < n; i += kB) {
        const SBend<T> s = reinterpret_cast<const SBend<T>*>(r)[i];
        int l[4] = {lo16(s.l01), hi16(s.l01), lo16(s.l23), hi16(s.l23)};
        Vec4<T> P[4] = {sX[l[0]], sX[l[1]], sX[l[2]], sX[l[3]]};
        T lbar = FIRST ? T(0) : mb[i], ab = FIRST || !AB ? T(0) : mb[n + i];
        if (bend_rev(P, st, i, n, s.th0, s.at, lbar, ab)) {
          sX[l[0]] = P[0]; sX[l[1]] = P[1]; sX[l[2]] = P[2]; sX[l[3]] = P[3];
        }
        mb[i] = lbar;
        if (AB) mb[n + i] = ab;
      }
      break;
    case 2:
      if constexpr (HEAVY)
      for (int i = tid; i < n; i += kB) {
        const STet<T>& s = reinterpret_cast<const STet<T>*>(r)[i];
        int l[4] = {lo16(s.l01), hi16(s.l01), lo16(s.l23), hi16(s.l23)};
        Vec4<T> P[4] = {sX[l[0]], sX[l[1]], sX[l[2]], sX[l[3]]};
        M3<T> B;
#pragma unroll
        for (int k = 0; k < 9; ++k) B.m[k / 3][k % 3] = s.B[k];
        T lbD = FIRST ? T(0) : mb[i], lbH = FIRST ? T(0) : mb[n + i];
        T ebD = FIRST ? T(0) : mb[2 * n + i], ebH = FIRST ? T(0) : mb[3 * n + i];
        T gb = FIRST ? T(0) : mb[4 * n + i];
        if (tet_rev(P, st + i, n, B, s.atD, s.atH, s.gam, lbD, lbH, ebD, ebH, gb)) {
          sX[l[0]] = P[0]; sX[l[1]] = P[1]; sX[l[2]] = P[2]; sX[l[3]] = P[3];
        }
        mb[i] = lbD; mb[n + i] = lbH; mb[2 * n + i] = ebD; mb[3 * n + i] = ebH; mb[4 * n + i] = gb;
      }
      break;
    case 4:
      if constexpr (HEAVY)
      for (int i = tid; i < n; i += kB) {
        const STri<T>& s = reinterpret_cast<const STri<T>*>(r)[i];
        int l[3] = {lo16(s.l01), hi16(s.l01), (int)s.l2};
        Vec4<T> P[3] = {sX[l[0]], sX[l[1]], sX[l[2]]};
        T B[4] = {s.B[0], s.B[1], s.B[2], s.B[3]}, at[4] = {s.at[0], s.at[1], s.at[2], s.at[3]};
        T lbar[3], ab[4];
#pragma unroll
        for (int c = 0; c < 3; ++c) lbar[c] = FIRST ? T(0) : mb[c * n + i];
#pragma unroll
        for (int c = 0; c < 4; ++c) ab[c] = FIRST ? T(0) : mb[(3 + c) * n + i];
        if (tri_rev(P, st, i, n, B, at, lbar, ab)) { sX[l[0]] = P[0]; sX[l[1]] = P[1]; sX[l[2]] = P[2]; }
#pragma unroll
        for (int c = 0; c < 3; ++c) mb[c * n + i] = lbar[c];
#pragma unroll
        for (int c = 0; c < 4; ++c) mb[(3 + c) * n + i] = ab[c];
      }
      break;
    case 5:
      if constexpr (HEAVY)
      for (int i = tid; i < n; i += kB) {
        const SBody<T> e = reinterpret_cast<const SBody<T>*>(r)[i];
        const int tri = D.bpair[e.j];
        T lbar = FIRST ? T(0) : mb[i];
        if (tri >= 0) {
          Vec4<T> P = sX[e.l];
          if (body_rev(P, st[i], D.bx, D.btri[tri], D.bc_tau, D.bc_at, lbar, D.bgrad)) sX[e.l] = P;
        }
        mb[i] = lbar;
      }
      break;
    default: {
      Vec4<T>* sam = reinterpret_cast<Vec4<T>*>(m);
      T* lbm = reinterpret_cast<T*>(sam + n);
      for (int i = tid; i < n; i += kB) {
        const int l = (int)reinterpret_cast<const SCon<T>*>(r)[i].l;
        Vec4<T> P = sX[l];
        T lbar = FIRST ? T(0) : lbm[i];
        Vec4<T> sa = FIRST ? Vec4<T>{T(0), T(0), T(0), T(0)} : sam[i];
        if (contact_rev(P, st[i], D.sph, lbar, sa)) sX[l] = P;
        lbm[i] = lbar; sam[i] = sa;
      }
      break;
    }
  }
}

// After the last reverse iteration of a substep (the forward's first): the
// FP64 parameter adjoints and the per-contact sphere adjoints leave the
// reverse state of patch p (each thread reads the items it wrote itself).
template <class T, bool HEAVY, bool AB>
__device__ __forceinline__ void group_rev_last(const Dev<T>& D, const GroupDev& G, int p, const int* cnt,
                                               const int* sty, const unsigned char* mul) {
  const int tid = threadIdx.x, kB = blockDim.x;
  const int* first = G.rec_first + (size_t)p * G.nset;
  const unsigned char* m = mul;
  for (int q = 0; q < G.nset; ++q) {
    const int n = cnt[q], ty = sty[q], jb = first[q];
    const T* mb = reinterpret_cast<const T*>(m);
    switch (ty) {
      case 0: if constexpr (AB) for (int i = tid; i < n; i += kB) D.d_acc[jb + i] += (double)mb[n + i]; break;
      case 1: if constexpr (AB) for (int i = tid; i < n; i += kB) D.b_acc[jb + i] += (double)mb[n + i]; break;
      case 2:
        if constexpr (HEAVY)
        for (int i = tid; i < n; i += kB) {
          D.t_acc[jb + i] += (double)mb[2 * n + i];
          D.t_acc[D.tr.n + jb + i] += (double)mb[3 * n + i];
          D.t_acc[2 * D.tr.n + jb + i] += (double)mb[4 * n + i];
        }
        break;
      case 4:
        if constexpr (HEAVY)
        for (int i = tid; i < n; i += kB) {
#pragma unroll
          for (int c = 0; c < 4; ++c) D.m_acc[(size_t)c * D.mr.n + jb + i] += (double)mb[(3 + c) * n + i];
        }
        break;
      case 5: break;   // body-vertex gradients were added during the reverse
      default: {
        const Vec4<T>* sam = reinterpret_cast<const Vec4<T>*>(m);
        for (int i = tid; i < n; i += kB) D.c_sacc[jb + i] = sam[i];
        break;
      }
    }
    m += al32((size_t)n * rmul_words(ty) * sizeof(T));
  }
}

// REPLAY (1, 2): the forward kept a snapshot of this launch's inputs (REC 2
// of k_group_fwd) instead of the record of every projection: the patch's
// positions go into a second LDS tile, the forward sets are replayed on it
// from the snapshot multipliers (group_sets_fwd, so every projection repeats
// the forward's arithmetic exactly) and write the record into LDS (with the
// entries staged, RL, or after the two tiles, REPLAY 2) or into this
// launch's scratch (REPLAY 1, at scratch + G.tpos[p]), where each thread
// reads back only the items it wrote.  AB false: the call asked for no
// distance or bending compliance gradient, so those adjoints are left out
// (fewer registers: a fifth wave per SIMD for the distance / bending groups).
template <class T, bool FIRST, bool LAST, bool RL, bool HEAVY, int REPLAY, bool AB = true>
__global__ __launch_bounds__(kBlock) void k_group_rev(Dev<T> D, GroupDev G, const char* __restrict__ img,
                                                      char* __restrict__ rmul, const char* __restrict__ tape_iter,
                                                      char* __restrict__ scratch) {
  extern __shared__ __align__(32) unsigned char smem[];
  __shared__ int cnt[kMaxGroupSets], sty[kMaxGroupSets];
  const int p = blockIdx.x, tid = threadIdx.x, kB = blockDim.x;
  const int v0 = G.pv_start[p], nv = G.pv_start[p + 1] - v0;
  stage_sets(G, p, cnt, sty);
  Vec4<T>* sX = reinterpret_cast<Vec4<T>*>(smem);
  size_t rbytes = 0, mbytes = 0, tbytes = 0;
  for (int q = 0; q < G.nset; ++q) {
    rbytes += al32((size_t)cnt[q] * rec_bytes<T>(sty[q]));
    mbytes += al32((size_t)cnt[q] * rmul_words(sty[q]) * sizeof(T));
    tbytes += al32((size_t)cnt[q] * tape_words(sty[q]) * sizeof(T));
  }
  const char* gimg = img + G.img[p];
  char* gmul = rmul + G.rmul[p];
  const char* gtap = REPLAY ? scratch + G.tpos[p] : tape_iter + G.tape_off + G.tpos[p];
  unsigned char* lrec = smem + al32((size_t)nv * sizeof(Vec4<T>));
  Vec4<T>* sP = REPLAY ? reinterpret_cast<Vec4<T>*>(lrec + (RL ? rbytes + mbytes + tbytes : 0)) : nullptr;
  // REPLAY 2: the replayed record in LDS after the two tiles
  unsigned char* ltap = lrec + al32((size_t)nv * sizeof(Vec4<T>));
  const unsigned char* rec = RL ? lrec : reinterpret_cast<const unsigned char*>(gimg);
  unsigned char* mul = RL ? lrec + rbytes : reinterpret_cast<unsigned char*>(gmul);
  const unsigned char* tap = RL ? lrec + rbytes + mbytes
                                : REPLAY == 2 ? ltap : reinterpret_cast<const unsigned char*>(gtap);
  const T* snx = REPLAY ? reinterpret_cast<const T*>(tape_iter + G.snap_x_off) + 3 * (size_t)v0 : nullptr;
  for (int i = tid; i < nv; i += kB) {
    const Vec4<T> xb = D.XB[G.pv[v0 + i]];   // adjoint and inverse mass
    sX[i] = xb;
    if (REPLAY) sP[i] = Vec4<T>{snx[3 * i], snx[3 * i + 1], snx[3 * i + 2], xb.w};
  }
  if (RL) {
    copy16(lrec, gimg, rbytes);
    if (!FIRST) copy16(lrec + rbytes, gmul, mbytes);   // the last iteration's reverse starts from zero
    if (!REPLAY) copy16(lrec + rbytes + mbytes, gtap, tbytes);
  }
  lds_barrier();
  if (REPLAY) {
    // the forward of iteration 0 (LAST here) started from lambda = 0
    unsigned char* lsn = reinterpret_cast<unsigned char*>(const_cast<char*>(tape_iter)) + G.snap_l_off +
                         (G.fmul[p] - G.fmul_lo);
    char* dst = RL ? reinterpret_cast<char*>(lrec + rbytes + mbytes)
                   : REPLAY == 2 ? reinterpret_cast<char*>(ltap) : scratch + G.tpos[p];
    group_sets_fwd<T, LAST, true, HEAVY, false>(D, G, cnt, sty, sP, rec, lsn, dst);
  }
  // walk the sets backwards: start past the last region
  const unsigned char* r = rec + rbytes;
  unsigned char* m = mul + mbytes;
  const unsigned char* t = tap + tbytes;
  for (int q = G.nset - 1; q >= 0; --q) {
    const int n = cnt[q], ty = sty[q];
    r -= al32((size_t)n * rec_bytes<T>(ty));
    m -= al32((size_t)n * rmul_words(ty) * sizeof(T));
    t -= al32((size_t)n * tape_words(ty) * sizeof(T));
    group_set_rev<T, FIRST, HEAVY, AB>(D, ty, n, r, m, t, sX);
    lds_barrier();
  }
  for (int i = tid; i < nv; i += kB) D.XB[G.pv[v0 + i]] = sX[i];
  if (!LAST) {
    if (RL) copy16(gmul, lrec + rbytes, mbytes);
    return;
  }
  // last reverse iteration of the substep: the parameter adjoints leave the state
  group_rev_last<T, HEAVY, AB>(D, G, p, cnt, sty, mul);
}

// copy the per-call compliances (alpha / h^2, the tet constants, a membrane's
// four at entries from at[4][n]) into the constant group image: pos[j] is
// the byte offset of constraint j's entry, -1 outside LDS groups
template <class T>
__global__ __launch_bounds__(kBlock) void k_group_fill(int type, int n, const long long* __restrict__ pos,
                                                       char* __restrict__ img, const T* __restrict__ at,
                                                       const T* __restrict__ atH, const T* __restrict__ gam) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n || pos[j] < 0) return;
  switch (type) {
    case 0: reinterpret_cast<SDist<T>*>(img + pos[j])->at = at[j]; break;
    case 1: reinterpret_cast<SBend<T>*>(img + pos[j])->at = at[j]; break;
    case 4: {
      STri<T>* f = reinterpret_cast<STri<T>*>(img + pos[j]);
#pragma unroll
      for (int c = 0; c < 4; ++c) f->at[c] = at[(size_t)c * n + j];
      break;
    }
    default: {
      STet<T>* f = reinterpret_cast<STet<T>*>(img + pos[j]);
      f->atD = at[j]; f->atH = atH[j]; f->gam = gam[j];
      break;
    }
  }
}

// ===================================================================== persistent program kernel

enum PhaseOp : int {
  OP_PREDICT = 0, OP_VELOCITY = 1, OP_REV_VELOCITY = 2, OP_REV_PREDICT = 3, OP_SPHERE = 4,
  OP_SET = 8,        // + type (0 dist, 1 bend, 2 tet, 3 contact, 4 membrane): forward projection of a set
  OP_SET_REV = 16,   // + type: reverse of a set
};
enum PhaseFlag : int { PF_FIRST = 1, PF_SECOND = 2 };   // SECOND = record (forward) or LAST (reverse)

struct Phase {
  int op, flags, begin, count;
  long long tape_off;   // byte offset of the set's record from the launch's record base, -1: none
};

// Per-launch arguments of one program run.
template <class T> struct RunArgs {
  char* tape;           // record base of this launch
  const T* f;           // external force of the frame, or null
  T* fbar;              // external-force adjoint of the frame, or null
  double* sph_out;      // FP64 sphere gradient, or null
  int record;           // forward: write the record where the phase has one
  unsigned* bar;        // barrier flags: kFlagStride words per block + release word (zero at launch)
  int* abort;           // set when a barrier wait runs out (bounded wait)
  unsigned spin_limit;  // polls before a barrier wait gives up
};

// Grid-wide barrier for a cooperative launch without read-modify-write
// contention: block b publishes the barrier's epoch in its own flag (one
// 128-byte line per block); block 0 waits for every flag (its threads poll
// disjoint flags in parallel), then publishes the epoch in the release word
// that the other blocks poll.  The agent-scope fences make each block's
// writes visible to the other XCDs before it arrives and drop stale cache
// lines after release.  Waits are bounded: past spin_limit polls a block
// records an abort and every block leaves at its next barrier.
constexpr int kFlagStride = 32;   // unsigned words between block flags (128 B)

__device__ __forceinline__ bool spin_until(const unsigned* p, unsigned epoch, int* abort, unsigned spin_limit) {
  unsigned polls = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
    if (++polls > spin_limit) {
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if ((polls & 63) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__device__ __forceinline__ bool grid_barrier(unsigned* flags, unsigned epoch, int* abort, unsigned spin_limit) {
  __shared__ int s_ok;
  unsigned* release = flags + (size_t)gridDim.x * kFlagStride;
  __syncthreads();
  if (threadIdx.x == 0) {
    s_ok = 1;
    __threadfence();
    __hip_atomic_store(flags + (size_t)blockIdx.x * kFlagStride, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    bool ok = true;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
      if (!spin_until(flags + (size_t)b * kFlagStride, epoch, abort, spin_limit)) { ok = false; break; }
    if (!ok) s_ok = 0;
    __syncthreads();
    if (threadIdx.x == 0 && s_ok) {
      __threadfence();
      __hip_atomic_store(release, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (threadIdx.x == 0) {
    if (!spin_until(release, epoch, abort, spin_limit)) s_ok = 0;
  }
  if (threadIdx.x == 0) __threadfence();
  __syncthreads();
  return s_ok != 0;
}

#define XPBD_GRID_LOOP(ITEM, TP)                                                                          \
  {                                                                                                       \
    const int stride = gridDim.x * kBlock;                                                                \
    const int base = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;                              \
    TP* tp = (TP*)(P.tape_off >= 0 ? R.tape + P.tape_off : nullptr);                                      \
    bool f1 = P.flags & PF_FIRST, f2 = P.flags & PF_SECOND;                                               \
    if (f1 && f2) { for (int t = base; t < P.count; t += stride) ITEM<T, true, true>(D, P.begin, P.count, t, tp); }   \
    else if (f1) { for (int t = base; t < P.count; t += stride) ITEM<T, true, false>(D, P.begin, P.count, t, tp); }   \
    else if (f2) { for (int t = base; t < P.count; t += stride) ITEM<T, false, true>(D, P.begin, P.count, t, tp); }   \
    else { for (int t = base; t < P.count; t += stride) ITEM<T, false, false>(D, P.begin, P.count, t, tp); }         \
  }

template <class T>
__global__ __launch_bounds__(kBlock) void k_program(Dev<T> D, const Phase* __restrict__ prog, int n_phases,
                                                    RunArgs<T> R) {
  __shared__ double sh[4][kBlock];
  unsigned epoch = 0;
  for (int p = 0; p < n_phases; ++p) {
    Phase P = prog[p];
    if (!R.record && P.op < OP_SET_REV && P.op >= OP_SET) P.flags &= ~PF_SECOND;
    if (P.op >= OP_SET && P.op < OP_SET_REV && !(P.flags & PF_SECOND)) P.tape_off = -1;
    switch (P.op) {
      case OP_PREDICT:
        for (int k = blockIdx.x * kBlock + threadIdx.x; k < D.V; k += gridDim.x * kBlock) predict_item(D, k, R.f);
        break;
      case OP_VELOCITY:
        for (int k = blockIdx.x * kBlock + threadIdx.x; k < D.V; k += gridDim.x * kBlock) velocity_item(D, k);
        break;
      case OP_REV_VELOCITY:
        for (int k = blockIdx.x * kBlock + threadIdx.x; k < D.V; k += gridDim.x * kBlock) rev_velocity_item(D, k);
        break;
      case OP_REV_PREDICT:
        for (int k = blockIdx.x * kBlock + threadIdx.x; k < D.V; k += gridDim.x * kBlock)
          rev_predict_item(D, k, R.fbar);
        break;
      case OP_SPHERE:
        if (blockIdx.x == 0 && R.sph_out)
          sphere_reduce_block<T, kBlock>(D.c_sacc, D.c_order, P.begin, P.count, R.sph_out, sh);
        break;
      case OP_SET + 0: XPBD_GRID_LOOP(dist_item, Vec4<T>) break;
      case OP_SET + 1: XPBD_GRID_LOOP(bend_item, Vec4<T>) break;
      case OP_SET + 2: XPBD_GRID_LOOP(tet_item, Vec4<T>) break;
      case OP_SET + 3: XPBD_GRID_LOOP(contact_item, Vec4<T>) break;
      case OP_SET + 4: XPBD_GRID_LOOP(tri_item, Vec4<T>) break;
      case OP_SET_REV + 0: XPBD_GRID_LOOP(dist_rev_item, const Vec4<T>) break;
      case OP_SET_REV + 1: XPBD_GRID_LOOP(bend_rev_item, const Vec4<T>) break;
      case OP_SET_REV + 2: XPBD_GRID_LOOP(tet_rev_item, const Vec4<T>) break;
      case OP_SET_REV + 3: XPBD_GRID_LOOP(contact_rev_item, const Vec4<T>) break;
      case OP_SET_REV + 4: XPBD_GRID_LOOP(tri_rev_item, const Vec4<T>) break;
      default: break;
    }
    if (p + 1 == n_phases) break;   // kernel end orders the last phase
    ++epoch;
    if (!grid_barrier(R.bar, epoch, R.abort, R.spin_limit)) return;
  }
}
#undef XPBD_GRID_LOOP

}  // namespace xpbd
