// Kernels of the implicit adjoint (Sec. 4.2, Eq. adjointXPBD, with the
// partial derivatives of Sec. 4.3): each substep's projection is taken as
// converged, x = y + M^-1 sum_j grad C_j lambda_j with lambda_j = -C_j /
// alpha~_j at the substep's end state, and its adjoint solves
//     (I - M^-1 K)^T w = xbar,   K = sum_j (lambda_j Hess C_j - grad C_j grad C_j^T / alpha~_j).
// With w = M y on the free vertices this is the symmetric system
// (M - K) y = xbar restricted to the free vertices, solved by preconditioned
// conjugate gradients in FP64.  The operator is applied matrix-free, one
// launch per independent set: no two constraints of a set share a vertex,
// so every constraint adds its 3x3 blocks' action to its own vertices
// without atomics.  Pinned vertices keep y = 0; their w is xbar + (K y).
#pragma once

#include "xpbd_kernels.hpp"

namespace xpbd {

using D4 = Vec4<double>;

__device__ __forceinline__ V3<double> d3(const D4& v) { return {v.x, v.y, v.z}; }
template <class T> __device__ __forceinline__ V3<double> pos(const Vec4<T>& v) {
  return {(double)v.x, (double)v.y, (double)v.z};
}
__device__ __forceinline__ void add3(D4& o, V3<double> a) { o.x += a.x; o.y += a.y; o.z += a.z; }

enum ImpMode {
  IMP_APPLY = 0,  // Q += -K P (every vertex of the constraint)
  IMP_DIAG = 1,   // Q += (grad C)^2 / alpha~ componentwise (Jacobi preconditioner)
  IMP_GRAD = 2,   // acc_j += (grad C_j . P) (-lambda_j / alpha~_j) / h^2
  IMP_BUILD = 3,  // store the constraint's block -lambda Hess C projected to PSD
  IMP_APPLY_PD = 4,  // Q += (N+ + g g^T / alpha~) P with the stored projected block N+
  IMP_DIAG_PD = 5    // Q += diag(N+) + g^2 / alpha~
};

// Positive-semidefinite part of a symmetric n x n matrix (row-major, in
// place, n <= 12): cyclic Jacobi rotations diagonalise it, eigenvalues below
// zero are dropped and the matrix is rebuilt from the rest.
__device__ inline void psd_part(int n, double* a) {
  double v[144];
  for (int i = 0; i < n * n; ++i) v[i] = 0.0;
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, all = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double x = a[i * n + j] * a[i * n + j];
        all += x;
        if (i != j) off += x;
      }
    if (!(off > 1e-30 * all)) break;
    for (int p = 0; p + 1 < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        // the rotation by phi with cot(2 phi) = (a_qq - a_pp) / (2 a_pq) zeroes a_pq
        const double th = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double x = a[k * n + p], y = a[k * n + q];
          a[k * n + p] = c * x - s * y;
          a[k * n + q] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = a[p * n + k], y = a[q * n + k];
          a[p * n + k] = c * x - s * y;
          a[q * n + k] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = v[k * n + p], y = v[k * n + q];
          v[k * n + p] = c * x - s * y;
          v[k * n + q] = s * x + c * y;
        }
      }
  }
  double ev[12];
  for (int k = 0; k < n; ++k) ev[k] = a[k * n + k] > 0.0 ? a[k * n + k] : 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc += v[i * n + k] * ev[k] * v[j * n + k];
      a[i * n + j] = acc;
    }
}

// Store -lambda Hess C projected to PSD for one row with nv vertices; the
// Hessian's columns come from Hessian-vector products with unit directions.
template <class HVP>
__device__ __forceinline__ void build_block(int nv, double lam, HVP hvp, double* out) {
  const int n = 3 * nv;
  double a[144];
  for (int col = 0; col < n; ++col) {
    V3<double> dir[4] = {}, hv[4] = {};
    const int k = col / 3, b = col % 3;
    if (b == 0) dir[k].x = 1.0; else if (b == 1) dir[k].y = 1.0; else dir[k].z = 1.0;
    hvp(dir, hv);
    for (int r = 0; r < nv; ++r) {
      a[(3 * r) * n + col] = -lam * hv[r].x;
      a[(3 * r + 1) * n + col] = -lam * hv[r].y;
      a[(3 * r + 2) * n + col] = -lam * hv[r].z;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) a[i * n + j] = a[j * n + i] = 0.5 * (a[i * n + j] + a[j * n + i]);
  psd_part(n, a);
  for (int i = 0; i < n * n; ++i) out[i] = a[i];
}

// y_k += (N+ P)_k + g_k (g . P) / at  (stored block N+)
__device__ __forceinline__ void apply_block(int nv, const int* vid, const double* nb, const V3<double>* g, double at,
                                            const D4* __restrict__ P, D4* __restrict__ Q) {
  const int n = 3 * nv;
  double pv[12];
  double s = 0.0;
  for (int k = 0; k < nv; ++k) {
    D4 p = P[vid[k]];
    pv[3 * k] = p.x; pv[3 * k + 1] = p.y; pv[3 * k + 2] = p.z;
    s += g[k].x * p.x + g[k].y * p.y + g[k].z * p.z;
  }
  for (int k = 0; k < nv; ++k) {
    double r[3];
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int l = 0; l < n; ++l) acc += nb[(3 * k + b) * n + l] * pv[l];
      r[b] = acc;
    }
    D4 q = Q[vid[k]];
    q.x += r[0] + g[k].x * s / at;
    q.y += r[1] + g[k].y * s / at;
    q.z += r[2] + g[k].z * s / at;
    Q[vid[k]] = q;
  }
}
__device__ __forceinline__ void diag_block(int nv, const int* vid, const double* nb, const V3<double>* g, double at,
                                           D4* __restrict__ Q) {
  const int n = 3 * nv;
  for (int k = 0; k < nv; ++k) {
    D4 q = Q[vid[k]];
    q.x += nb[(3 * k) * n + 3 * k] + g[k].x * g[k].x / at;
    q.y += nb[(3 * k + 1) * n + 3 * k + 1] + g[k].y * g[k].y / at;
    q.z += nb[(3 * k + 2) * n + 3 * k + 2] + g[k].z * g[k].z / at;
    Q[vid[k]] = q;
  }
}

// one constraint row with n vertices: value C, gradient g, stiffness at
template <int MODE>
__device__ __forceinline__ void imp_row(int n, const int* vid, double C, double at, const V3<double>* g,
                                        const V3<double>* hv, const D4* __restrict__ P, D4* __restrict__ Q,
                                        double* acc, double ih2) {
  const double lam = -C / at;
  if (MODE == IMP_DIAG) {
    for (int k = 0; k < n; ++k) {
      D4 q = Q[vid[k]];
      q.x += g[k].x * g[k].x / at; q.y += g[k].y * g[k].y / at; q.z += g[k].z * g[k].z / at;
      Q[vid[k]] = q;
    }
    return;
  }
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += dot(g[k], d3(P[vid[k]]));
  if (MODE == IMP_GRAD) {
    *acc += s * (-lam / at) * ih2;
    return;
  }
  for (int k = 0; k < n; ++k) {
    D4 q = Q[vid[k]];
    add3(q, (-lam) * hv[k] + (s / at) * g[k]);
    Q[vid[k]] = q;
  }
}

// one row (constraint, or one of a tet's two projections) in any mode
template <int MODE, class HVP>
__device__ __forceinline__ void imp_any(int nv, const int* vid, double C, double at, const V3<double>* g, HVP hvp,
                                        const D4* __restrict__ P, D4* __restrict__ Q, double* acc, double* nb,
                                        double ih2) {
  const double lam = -C / at;
  if (MODE == IMP_BUILD) {
    build_block(nv, lam, hvp, nb);
  } else if (MODE == IMP_APPLY_PD) {
    apply_block(nv, vid, nb, g, at, P, Q);
  } else if (MODE == IMP_DIAG_PD) {
    diag_block(nv, vid, nb, g, at, Q);
  } else {
    V3<double> gb[4] = {}, hv[4] = {};
    if (MODE == IMP_APPLY) {
      for (int k = 0; k < nv; ++k) gb[k] = d3(P[vid[k]]);
      hvp(gb, hv);
    }
    imp_row<MODE>(nv, vid, C, at, g, hv, P, Q, acc, ih2);
  }
}

// NB: stored projected blocks of this constraint type (per internal index:
// 36 doubles per distance, 144 per hinge, 2 x 144 per tet, 9 per contact)
template <class T, int TY, int MODE>
__global__ __launch_bounds__(kBlock) void k_imp_set(Dev<T> D, int begin, int count, const Vec4<T>* __restrict__ XE,
                                                    const D4* __restrict__ P, D4* __restrict__ Q, double ih2,
                                                    int* __restrict__ bad, double* __restrict__ NB) {
  const int t = thread_item(count);
  if (t < 0) return;
  const int j = begin + t;
  if (TY == 0) {
    const int2 e = D.d_idx[j];
    const int vid[2] = {e.x, e.y};
    DistEval<double> ev = dist_eval(pos(XE[e.x]) - pos(XE[e.y]), (double)D.d_rest[j]);
    if (!ev.ok) return;
    const double at = (double)D.d_at[j];
    if (!(at > 0.0)) { *bad = 1; return; }
    V3<double> g[2] = {ev.n, -ev.n};
    auto hvp = [&](const V3<double>* gb, V3<double>* hv) {
      V3<double> d = gb[0] - gb[1];
      hv[0] = (1.0 / ev.len) * (d - dot(d, ev.n) * ev.n);
      hv[1] = -hv[0];
    };
    imp_any<MODE>(2, vid, ev.C, at, g, hvp, P, Q, D.d_acc + j, NB ? NB + (size_t)j * 36 : nullptr, ih2);
  } else if (TY == 1) {
    const int4 q = D.b_idx[j];
    const int vid[4] = {q.x, q.y, q.z, q.w};
    V3<double> x0 = pos(XE[q.x]);
    V3<double> e = pos(XE[q.y]) - x0, a = pos(XE[q.z]) - x0, b = pos(XE[q.w]) - x0;
    BendEval<double> ev = bend_eval(e, a, b, (double)D.b_th0[j]);
    if (!ev.ok) return;
    const double at = (double)D.b_at[j];
    if (!(at > 0.0)) { *bad = 1; return; }
    auto hvp = [&](const V3<double>* gb, V3<double>* hv) { bend_hvp(e, a, b, gb, hv); };
    imp_any<MODE>(4, vid, ev.C, at, ev.g, hvp, P, Q, D.b_acc + j, NB ? NB + (size_t)j * 144 : nullptr, ih2);
  } else if (TY == 2) {
    if (MODE == IMP_GRAD) return;   // the tets' parameter gradient is not produced by this adjoint
    const TetRec<T>& R = D.tr;
    const int4 q = R.idx[j];
    const int vid[4] = {q.x, q.y, q.z, q.w};
    V3<double> x0 = pos(XE[q.x]);
    const V3<double> dd[3] = {pos(XE[q.y]) - x0, pos(XE[q.z]) - x0, pos(XE[q.w]) - x0};
    M3<T> Bt = load_B(R.B, R.n, j);
    M3<double> B;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) B.m[r][c] = (double)Bt.m[r][c];
    // deviatoric and hydrostatic rows, both at the end state
    TetEval<double> evD = tet_dev_eval(dd, B);
    if (evD.ok) {
      const double at = (double)R.atD[j];
      if (!(at > 0.0)) { *bad = 1; return; }
      auto hvp = [&](const V3<double>* gb, V3<double>* hv) { tet_dev_hvp(evD, B, gb, hv); };
      imp_any<MODE>(4, vid, evD.C, at, evD.g, hvp, P, Q, nullptr, NB ? NB + (size_t)j * 288 : nullptr, ih2);
    }
    TetEval<double> evH = tet_hyd_eval(dd, B, (double)R.gamma[j]);
    const double at = (double)R.atH[j];
    if (!(at > 0.0)) { *bad = 1; return; }
    auto hvp = [&](const V3<double>* gb, V3<double>* hv) { tet_hyd_hvp(evH, B, gb, hv); };
    imp_any<MODE>(4, vid, evH.C, at, evH.g, hvp, P, Q, nullptr, NB ? NB + (size_t)j * 288 + 144 : nullptr, ih2);
  } else {
    if (MODE == IMP_GRAD) return;
    const int v = D.c_vid[j];
    const int vid[1] = {v};
    const V3<double> c = {(double)D.sph.cx, (double)D.sph.cy, (double)D.sph.cz};
    ContactEval<double> ev = contact_eval(pos(XE[v]) - c, (double)D.sph.R, (double)D.sph.tau);
    if (!ev.ok || !(ev.C < 0.0)) return;
    const double at = (double)D.sph.at;
    if (!(at > 0.0)) { *bad = 1; return; }
    V3<double> g[1] = {ev.n};
    auto hvp = [&](const V3<double>* gb, V3<double>* hv) {
      hv[0] = (1.0 / ev.d) * (gb[0] - dot(gb[0], ev.n) * ev.n);
    };
    imp_any<MODE>(1, vid, ev.C, at, g, hvp, P, Q, nullptr, NB ? NB + (size_t)j * 9 : nullptr, ih2);
  }
}

// Q = M P on free vertices (M = 1 / w), 0 on pinned ones
template <class T>
__global__ __launch_bounds__(kBlock) void k_imp_mass(const Vec4<T>* __restrict__ XB, const D4* __restrict__ P,
                                                     D4* __restrict__ Q, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  double w = (double)XB[k].w;
  D4 p = P[k];
  Q[k] = w > 0.0 ? D4{p.x / w, p.y / w, p.z / w, 0.0} : D4{0.0, 0.0, 0.0, 0.0};
}

// b = xbar on free vertices (0 on pinned), y = 0, r = b
template <class T>
__global__ __launch_bounds__(kBlock) void k_imp_rhs(const Vec4<T>* __restrict__ XB, D4* __restrict__ Bv,
                                                    D4* __restrict__ Y, D4* __restrict__ R, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  Vec4<T> x = XB[k];
  D4 b = x.w > T(0) ? D4{(double)x.x, (double)x.y, (double)x.z, 0.0} : D4{0.0, 0.0, 0.0, 0.0};
  Bv[k] = b;
  R[k] = b;
  Y[k] = D4{0.0, 0.0, 0.0, 0.0};
}

// deterministic partial sums of a . b (b = null: a . a) over the free
// vertices, or of a . (b / diag) when diag is given
__global__ __launch_bounds__(kBlock) void k_imp_dot(const D4* __restrict__ a, const D4* __restrict__ b,
                                                    const D4* __restrict__ diag, int n, double* __restrict__ part) {
  __shared__ double sh[kBlock];
  int k = blockIdx.x * kBlock + threadIdx.x;
  double s = 0.0;
  if (k < n) {
    D4 x = a[k], y = b ? b[k] : a[k];
    if (diag) {
      D4 dg = diag[k];
      if (dg.x > 0.0) s += x.x * y.x / dg.x;
      if (dg.y > 0.0) s += x.y * y.y / dg.y;
      if (dg.z > 0.0) s += x.z * y.z / dg.z;
    } else {
      s = x.x * y.x + x.y * y.y + x.z * y.z;
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

// diag = M + accumulated (grad C)^2 / alpha~ on free vertices, 0 on pinned
// ones (the zero marks them for the other CG kernels)
template <class T>
__global__ __launch_bounds__(kBlock) void k_imp_diag(const Vec4<T>* __restrict__ XB, D4* __restrict__ DG, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  double w = (double)XB[k].w;
  D4 d = DG[k];
  DG[k] = w > 0.0 ? D4{d.x + 1.0 / w, d.y + 1.0 / w, d.z + 1.0 / w, 0.0} : D4{0.0, 0.0, 0.0, 0.0};
}

// p = r / diag + beta p (free vertices; pinned stay 0)
__global__ __launch_bounds__(kBlock) void k_imp_dir(double beta, const D4* __restrict__ R, const D4* __restrict__ DG,
                                                    D4* __restrict__ P, int n, int first) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  D4 r = R[k], dg = DG[k], p = first ? D4{0.0, 0.0, 0.0, 0.0} : P[k];
  D4 z = {dg.x > 0.0 ? r.x / dg.x : 0.0, dg.y > 0.0 ? r.y / dg.y : 0.0, dg.z > 0.0 ? r.z / dg.z : 0.0, 0.0};
  P[k] = D4{z.x + beta * p.x, z.y + beta * p.y, z.z + beta * p.z, 0.0};
}

// The CG loop keeps its scalars on the device, so a batch of iterations runs
// without the host: slot CG_RZ r.z, CG_PQ p.q, CG_RR r.r, CG_RZ2 the next
// r.z, CG_ALPHA, CG_BETA, CG_REL the relative residual |r| / |b|; state[0]
// is CG_RUN until the solve stops (converged, p.Ap <= 0, or the iteration
// limit), after which every step kernel leaves y, r and p as they are;
// state[1] counts the iterations taken.  Each scalar is the same FP64
// expression the host loop would evaluate, in the same order.
enum CgSlot { CG_RZ = 0, CG_PQ, CG_RR, CG_RZ2, CG_ALPHA, CG_BETA, CG_REL, CG_NSLOT };
enum CgState { CG_RUN = 0, CG_CONVERGED = 1, CG_INDEFINITE = 2, CG_LIMIT = 3 };

__global__ void k_cg_start(double* __restrict__ cg, int* __restrict__ state) {
  state[0] = CG_RUN;
  state[1] = 0;
  cg[CG_REL] = 1.0;
}

// alpha = r.z / p.q, or stop when the system is not positive definite
__global__ void k_cg_alpha(double* __restrict__ cg, int* __restrict__ state) {
  if (state[0] != CG_RUN) return;
  const double pq = cg[CG_PQ];
  if (!(pq > 0.0)) {
    state[0] = CG_INDEFINITE;
    return;
  }
  cg[CG_ALPHA] = cg[CG_RZ] / pq;
}

// one iteration done: stop when |r| / |b| <= tol or at the iteration limit
__global__ void k_cg_check(double* __restrict__ cg, int* __restrict__ state, double bn, double tol, int max_it) {
  if (state[0] != CG_RUN) return;
  state[1] += 1;
  const double rel = sqrt(cg[CG_RR]) / bn;
  cg[CG_REL] = rel;
  if (rel <= tol) state[0] = CG_CONVERGED;
  else if (state[1] >= max_it) state[0] = CG_LIMIT;
}

// beta = (next r.z) / r.z, and the next r.z becomes r.z
__global__ void k_cg_beta(double* __restrict__ cg, const int* __restrict__ state) {
  if (state[0] != CG_RUN) return;
  cg[CG_BETA] = cg[CG_RZ2] / cg[CG_RZ];
  cg[CG_RZ] = cg[CG_RZ2];
}

// y += alpha p, r -= alpha q (free vertices) and p = r / diag + beta p, with
// alpha and beta read from the device, doing nothing once the solve has
// stopped
__global__ __launch_bounds__(kBlock) void k_cg_axpy2(const double* __restrict__ cg, const int* __restrict__ state,
                                                     const D4* __restrict__ P, const D4* __restrict__ Q,
                                                     const D4* __restrict__ DG, D4* __restrict__ Y,
                                                     D4* __restrict__ R, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (state[0] != CG_RUN || k >= n || !(DG[k].x > 0.0)) return;
  const double alpha = cg[CG_ALPHA];
  D4 p = P[k], q = Q[k], y = Y[k], r = R[k];
  y.x += alpha * p.x; y.y += alpha * p.y; y.z += alpha * p.z;
  r.x -= alpha * q.x; r.y -= alpha * q.y; r.z -= alpha * q.z;
  Y[k] = y;
  R[k] = r;
}

__global__ __launch_bounds__(kBlock) void k_cg_dir(const double* __restrict__ cg, const int* __restrict__ state,
                                                   const D4* __restrict__ R, const D4* __restrict__ DG,
                                                   D4* __restrict__ P, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (state[0] != CG_RUN || k >= n) return;
  const double beta = cg[CG_BETA];
  D4 r = R[k], dg = DG[k], p = P[k];
  D4 z = {dg.x > 0.0 ? r.x / dg.x : 0.0, dg.y > 0.0 ? r.y / dg.y : 0.0, dg.z > 0.0 ? r.z / dg.z : 0.0, 0.0};
  P[k] = D4{z.x + beta * p.x, z.y + beta * p.y, z.z + beta * p.z, 0.0};
}

// After the solve (Q = (M - K) y on free vertices, -(K y) on pinned ones):
//   w = M y (free), w = xbar + K y (pinned);  xbar_prev = -vbar / h;
//   vbar_mid = h w (free), fbar += h w_inv vbar_mid;  vbar = vbar_mid;  xbar = w + xbar_prev
template <class T>
__global__ __launch_bounds__(kBlock) void k_imp_finish(Vec4<T>* __restrict__ XB, Vec4<T>* __restrict__ VB,
                                                       const D4* __restrict__ Y, const D4* __restrict__ Q,
                                                       T* __restrict__ fbar, double h, int n) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  Vec4<T> xb = XB[k], vb = VB[k];
  const double wi = (double)xb.w;
  D4 y = Y[k];
  V3<double> w, vm = {0.0, 0.0, 0.0};
  if (wi > 0.0) {
    w = {y.x / wi, y.y / wi, y.z / wi};
    vm = h * w;
    if (fbar) {
      fbar[3 * k] += (T)(h * wi * vm.x);
      fbar[3 * k + 1] += (T)(h * wi * vm.y);
      fbar[3 * k + 2] += (T)(h * wi * vm.z);
    }
  } else {
    D4 q = Q[k];
    w = {(double)xb.x - q.x, (double)xb.y - q.y, (double)xb.z - q.z};
  }
  XB[k] = Vec4<T>{(T)(w.x - (double)vb.x / h), (T)(w.y - (double)vb.y / h), (T)(w.z - (double)vb.z / h), xb.w};
  VB[k] = Vec4<T>{(T)vm.x, (T)vm.y, (T)vm.z, T(0)};
}

}  // namespace xpbd
