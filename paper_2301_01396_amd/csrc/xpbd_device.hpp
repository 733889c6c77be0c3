// Device-side constraint math for the XPBD projections and their adjoints.
//
// Every constraint is evaluated from vertex *differences* only (edge
// vector, hinge/wing offsets, tet edge matrix), so the forward kernels can
// record exactly those differences and the reverse kernels recompute
// bit-identical C, grad C and dlambda from the record.
//
// Gradients are closed forms; Hessian-vector products (needed by the
// adjoint, the dJ/dx and d gradC/dx terms of Sec. 4.3) are closed forms for
// distance, contact and tets and, for the dihedral angle, the directional
// derivative of its closed-form gradient taken with dual numbers.
#pragma once
#include <hip/hip_runtime.h>

namespace xpbd {

template <class T> struct alignas(sizeof(T) * 4) Vec4 { T x, y, z, w; };
template <class T> struct alignas(sizeof(T) * 2) Vec2 { T x, y; };

template <class S> struct V3 { S x, y, z; };

template <class S> __device__ __forceinline__ V3<S> mk(S a, S b, S c) { return V3<S>{a, b, c}; }
template <class S> __device__ __forceinline__ V3<S> operator+(V3<S> a, V3<S> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> __device__ __forceinline__ V3<S> operator-(V3<S> a, V3<S> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> __device__ __forceinline__ V3<S> operator-(V3<S> a) { return {-a.x, -a.y, -a.z}; }
template <class S, class U> __device__ __forceinline__ V3<S> operator*(U s, V3<S> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class S> __device__ __forceinline__ S dot(V3<S> a, V3<S> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> __device__ __forceinline__ V3<S> cross(V3<S> a, V3<S> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> __device__ __forceinline__ V3<T> xyz(const Vec4<T>& v) { return {v.x, v.y, v.z}; }

// ----------------------------------------------------------------- duals
// (value, directional derivative) pairs for the dihedral Hessian-vector product
template <class T> struct Dual { T v, d; };
template <class T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class T> __device__ __forceinline__ Dual<T> operator*(T s, Dual<T> a) { return {s * a.v, s * a.d}; }
template <class T> __device__ __forceinline__ Dual<T> dsqrt(Dual<T> a) {
  T r = sqrt(a.v);
  return {r, T(0.5) * a.d * (T(1) / r)};   // 1/r is the quotient the gradient forms next
}
template <class T> __device__ __forceinline__ T dsqrt(T a) { return sqrt(a); }
template <class T> __device__ __forceinline__ T val(T a) { return a; }
template <class T> __device__ __forceinline__ T val(Dual<T> a) { return a.v; }
template <class T> __device__ __forceinline__ T scal(T s, T) { return s; }

// ----------------------------------------------------------------- distance
// C = |r| - L, grad_i = n, grad_j = -n (n = r/|r|).
template <class T> struct DistEval { T C, len, inv; V3<T> n; bool ok; };
template <class T> __device__ __forceinline__ DistEval<T> dist_eval(V3<T> r, T L) {
  DistEval<T> e;
  T l2 = dot(r, r);
  e.ok = l2 > T(0);
  e.len = sqrt(l2);
  e.inv = T(1) / e.len;
  e.n = e.inv * r;
  e.C = e.len - L;
  return e;
}

// ----------------------------------------------------------------- dihedral
// e = x1 - x0, a = x2 - x0, b = x3 - x0;  n1 = e x a, n2 = b x e;
// theta = atan2(((n1 x n2) . e)/|e|, n1 . n2).
// grad x2 = -|e| n1/|n1|^2, grad x3 = -|e| n2/|n2|^2,
// grad x1 = (a.e/|e|) n1/|n1|^2 + (b.e/|e|) n2/|n2|^2, grad x0 = -(sum).
template <class S> __device__ __forceinline__ S one_over(S x) { return S(1) / x; }
template <class T> __device__ __forceinline__ Dual<T> one_over(Dual<T> x) {
  T r = T(1) / x.v;
  return {r, -x.d * r * r};
}
template <class S> __device__ __forceinline__ void bend_gradient(V3<S> e, V3<S> a, V3<S> b, V3<S> g[4]) {
  V3<S> n1 = cross(e, a), n2 = cross(b, e);
  S le = dsqrt(dot(e, e));
  S r1 = one_over(S(dot(n1, n1))), r2 = one_over(S(dot(n2, n2))), rl = one_over(le);
  V3<S> s1 = {n1.x * r1, n1.y * r1, n1.z * r1};
  V3<S> s2 = {n2.x * r2, n2.y * r2, n2.z * r2};
  S c1 = dot(a, e) * rl, c2 = dot(b, e) * rl;
  g[2] = {-(le * s1.x), -(le * s1.y), -(le * s1.z)};
  g[3] = {-(le * s2.x), -(le * s2.y), -(le * s2.z)};
  g[1] = {c1 * s1.x + c2 * s2.x, c1 * s1.y + c2 * s2.y, c1 * s1.z + c2 * s2.z};
  g[0] = -(g[1] + g[2] + g[3]);
}
template <class T> struct BendEval { T C; V3<T> g[4]; bool ok; };
template <class T> __device__ __forceinline__ BendEval<T> bend_eval(V3<T> e, V3<T> a, V3<T> b, T theta0) {
  BendEval<T> r;
  V3<T> n1 = cross(e, a), n2 = cross(b, e);
  T le2 = dot(e, e), q1 = dot(n1, n1), q2 = dot(n2, n2);
  r.ok = le2 > T(0) && q1 > T(0) && q2 > T(0);
  T le = sqrt(le2);
  T y = dot(cross(n1, n2), e) * (T(1) / le);   // 1/|e| is the quotient the gradient forms too
  T x = dot(n1, n2);
  r.C = atan2(y, x) - theta0;
  bend_gradient<T>(e, a, b, r.g);
  return r;
}
// Hessian of theta times gbar: directional derivative of the gradient along
// (e, a, b) moved by (gbar1 - gbar0, gbar2 - gbar0, gbar3 - gbar0).
template <class T> __device__ __forceinline__ void bend_hvp(V3<T> e, V3<T> a, V3<T> b, const V3<T> gb[4], V3<T> hv[4]) {
  V3<T> de = gb[1] - gb[0], da = gb[2] - gb[0], db = gb[3] - gb[0];
  using D = Dual<T>;
  V3<D> E = {D{e.x, de.x}, D{e.y, de.y}, D{e.z, de.z}};
  V3<D> A = {D{a.x, da.x}, D{a.y, da.y}, D{a.z, da.z}};
  V3<D> B = {D{b.x, db.x}, D{b.y, db.y}, D{b.z, db.z}};
  V3<D> g[4];
  bend_gradient<D>(E, A, B, g);
  for (int k = 0; k < 4; ++k) hv[k] = {g[k].x.d, g[k].y.d, g[k].z.d};
}

// ----------------------------------------------------------------- Neo-Hookean tet
// F = Ds B with Ds columns d1, d2, d3 (= x1-x0, x2-x0, x3-x0), B = Dm^-1.
template <class T> struct M3 { T m[3][3]; };   // m[row][col]

template <class T> __device__ __forceinline__ M3<T> mul_DsB(const V3<T> d[3], const M3<T>& B) {
  M3<T> F;
  const T ds[3][3] = {{d[0].x, d[1].x, d[2].x}, {d[0].y, d[1].y, d[2].y}, {d[0].z, d[1].z, d[2].z}};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) F.m[r][c] = ds[r][0] * B.m[0][c] + ds[r][1] * B.m[1][c] + ds[r][2] * B.m[2][c];
  return F;
}
// vertex gradients from dC/dF: grad x_{k+1} = column k of P B^T, grad x0 = -sum
template <class T> __device__ __forceinline__ void grads_from_P(const M3<T>& P, const M3<T>& B, V3<T> g[4]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T c[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) c[r] = P.m[r][0] * B.m[k][0] + P.m[r][1] * B.m[k][1] + P.m[r][2] * B.m[k][2];
    g[k + 1] = {c[0], c[1], c[2]};
  }
  g[0] = -(g[1] + g[2] + g[3]);
}
template <class T> __device__ __forceinline__ V3<T> col(const M3<T>& F, int c) { return {F.m[0][c], F.m[1][c], F.m[2][c]}; }

template <class T> struct TetEval { T C; V3<T> g[4]; M3<T> F; bool ok; };
// deviatoric: C_D = |F|_F, dC/dF = F / C_D
template <class T> __device__ __forceinline__ TetEval<T> tet_dev_eval(const V3<T> d[3], const M3<T>& B) {
  TetEval<T> r;
  r.F = mul_DsB(d, B);
  T s = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += r.F.m[i][j] * r.F.m[i][j];
  r.ok = s > T(0);
  r.C = sqrt(s);
  T inv = T(1) / r.C;
  M3<T> P;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) P.m[i][j] = inv * r.F.m[i][j];
  grads_from_P(P, B, r.g);
  return r;
}
// hydrostatic: C_H = det F - gamma, dC/dF = cof F = [f1 x f2, f2 x f0, f0 x f1]
template <class T> __device__ __forceinline__ TetEval<T> tet_hyd_eval(const V3<T> d[3], const M3<T>& B, T gamma) {
  TetEval<T> r;
  r.F = mul_DsB(d, B);
  V3<T> f0 = col(r.F, 0), f1 = col(r.F, 1), f2 = col(r.F, 2);
  V3<T> c0 = cross(f1, f2), c1 = cross(f2, f0), c2 = cross(f0, f1);
  r.C = dot(f0, c0) - gamma;
  r.ok = true;
  M3<T> P;
  P.m[0][0] = c0.x; P.m[1][0] = c0.y; P.m[2][0] = c0.z;
  P.m[0][1] = c1.x; P.m[1][1] = c1.y; P.m[2][1] = c1.z;
  P.m[0][2] = c2.x; P.m[1][2] = c2.y; P.m[2][2] = c2.z;
  grads_from_P(P, B, r.g);
  return r;
}
// Z = dF along gbar:  Z = [gb1 - gb0, gb2 - gb0, gb3 - gb0] B
template <class T> __device__ __forceinline__ M3<T> tet_dF(const V3<T> gb[4], const M3<T>& B) {
  V3<T> d[3] = {gb[1] - gb[0], gb[2] - gb[0], gb[3] - gb[0]};
  return mul_DsB(d, B);
}
template <class T> __device__ __forceinline__ void tet_dev_hvp(const TetEval<T>& e, const M3<T>& B, const V3<T> gb[4], V3<T> hv[4]) {
  M3<T> Z = tet_dF(gb, B);
  T fz = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) fz += e.F.m[i][j] * Z.m[i][j];
  T inv = T(1) / e.C;
  T k = fz * inv * inv;
  M3<T> Y;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Y.m[i][j] = (Z.m[i][j] - k * e.F.m[i][j]) * inv;
  grads_from_P(Y, B, hv);
}
template <class T> __device__ __forceinline__ void tet_hyd_hvp(const TetEval<T>& e, const M3<T>& B, const V3<T> gb[4], V3<T> hv[4]) {
  M3<T> Z = tet_dF(gb, B);
  V3<T> f0 = col(e.F, 0), f1 = col(e.F, 1), f2 = col(e.F, 2);
  V3<T> z0 = col(Z, 0), z1 = col(Z, 1), z2 = col(Z, 2);
  V3<T> y0 = cross(z1, f2) + cross(f1, z2);
  V3<T> y1 = cross(z2, f0) + cross(f2, z0);
  V3<T> y2 = cross(z0, f1) + cross(f0, z1);
  M3<T> Y;
  Y.m[0][0] = y0.x; Y.m[1][0] = y0.y; Y.m[2][0] = y0.z;
  Y.m[0][1] = y1.x; Y.m[1][1] = y1.y; Y.m[2][1] = y1.z;
  Y.m[0][2] = y2.x; Y.m[1][2] = y2.y; Y.m[2][2] = y2.z;
  grads_from_P(Y, B, hv);
}

// ----------------------------------------------------------------- sphere contact
// C = |x - c| - R - tau, grad = n = (x - c)/|x - c|
template <class T> struct ContactEval { T C, d; V3<T> n; bool ok; };
template <class T> __device__ __forceinline__ ContactEval<T> contact_eval(V3<T> r, T R, T tau) {
  ContactEval<T> e;
  T d2 = dot(r, r);
  e.ok = d2 > T(0);
  e.d = sqrt(d2);
  T inv = T(1) / e.d;
  e.n = inv * r;
  e.C = e.d - R - tau;
  return e;
}

// Map a launch's block index to the logical tile so that consecutive tiles
// land on the same XCD (blocks are dealt to the 8 XCDs round-robin), which
// keeps neighbouring vertices in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  int q = nb >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

}  // namespace xpbd
