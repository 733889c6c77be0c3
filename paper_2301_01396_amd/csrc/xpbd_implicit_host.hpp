// Host side of the implicit adjoint (xpbd_adjoint_implicit in
// include/xpbd.h): per frame in reverse, the frame's substep end states are
// recomputed from its checkpoint; per substep in reverse, the symmetric
// system (M - K) y = xbar on the free vertices is solved by Jacobi-
// preconditioned conjugate gradients in FP64 with a matrix-free operator
// (one launch per independent set), then the vertex, velocity, force and
// compliance adjoints are updated from the solution.  Included once, at the
// end of xpbd.hip.
#pragma once

#include "xpbd_implicit_kernels.hpp"

namespace {

template <class T> struct ImpOps {
  using V4 = Vec4<T>;

  struct Work {
    V4* XS;       // [S][V] end state of each substep of the frame
    D4 *B, *Y, *R, *P, *Q, *DG;
    double* part; // [nblocks(V)]
    double* sum;  // [1]
    int* bad;     // [1]
    double* cg;   // [CG_NSLOT] scalars of the CG loop
    int* cgs;     // [2] CG state and iterations taken
    double* nb[4];  // projected blocks per constraint type (PD projection only)
  };

  static size_t block_doubles(xpbd_ctx c, int ty) {
    switch (ty) {
      case XPBD_DIST: return (size_t)c->n_dist * 36;
      case XPBD_BEND: return (size_t)c->n_bend * 144;
      case XPBD_TET: return (size_t)c->n_tet * 288;
      default: return (size_t)c->n_contact * 9;
    }
  }

  static Work work(xpbd_ctx c, bool pd) {
    const size_t V = (size_t)c->V, nb = nblocks(V);
    size_t need = align256((size_t)c->S * V * sizeof(V4)) + 6 * align256(V * sizeof(D4)) +
                  align256(nb * sizeof(double)) + 4 * 256;
    if (pd)
      for (int ty = 0; ty < 4; ++ty) need += align256(block_doubles(c, ty) * sizeof(double));
    if (c->imp_cap < need) {
      c->release(c->imp_buf);
      c->imp_cap = 0;
      c->imp_buf = c->alloc(need);
      c->imp_cap = need;
    }
    char* p = (char*)c->imp_buf;
    Work w;
    auto take = [&](size_t b) { char* q = p; p += align256(b); return q; };
    w.XS = (V4*)take((size_t)c->S * V * sizeof(V4));
    w.B = (D4*)take(V * sizeof(D4));
    w.Y = (D4*)take(V * sizeof(D4));
    w.R = (D4*)take(V * sizeof(D4));
    w.P = (D4*)take(V * sizeof(D4));
    w.Q = (D4*)take(V * sizeof(D4));
    w.DG = (D4*)take(V * sizeof(D4));
    w.part = (double*)take(nb * sizeof(double));
    w.sum = (double*)take(sizeof(double));
    w.bad = (int*)take(sizeof(int));
    w.cg = (double*)take(CG_NSLOT * sizeof(double));
    w.cgs = (int*)take(2 * sizeof(int));
    for (int ty = 0; ty < 4; ++ty) w.nb[ty] = pd && block_doubles(c, ty) ? (double*)take(block_doubles(c, ty) * sizeof(double)) : nullptr;
    return w;
  }

  template <int MODE>
  static void sets(xpbd_ctx c, const Dev<T>& D, const V4* XE, const D4* P, D4* Q, double ih2, int* bad,
                   const Work& w, hipStream_t st) {
    // the projected blocks are built with one thread per constraint and a
    // 12 x 12 eigen-decomposition each: smaller workgroups
    const int bs = MODE == IMP_BUILD ? 64 : kBlock;
    for (const SetInfo& si : c->sets) {
      if (si.count == 0) continue;
      if (MODE == IMP_GRAD && (si.type == XPBD_TET || si.type == XPBD_CONTACT)) continue;
      unsigned nb = nblocks(si.count, bs);
      double* NB = w.nb[si.type];
      switch (si.type) {
        case XPBD_DIST:
          k_imp_set<T, 0, MODE><<<nb, bs, 0, st>>>(D, si.begin, si.count, XE, P, Q, ih2, bad, NB);
          break;
        case XPBD_BEND:
          k_imp_set<T, 1, MODE><<<nb, bs, 0, st>>>(D, si.begin, si.count, XE, P, Q, ih2, bad, NB);
          break;
        case XPBD_TET:
          k_imp_set<T, 2, MODE><<<nb, bs, 0, st>>>(D, si.begin, si.count, XE, P, Q, ih2, bad, NB);
          break;
        default:
          k_imp_set<T, 3, MODE><<<nb, bs, 0, st>>>(D, si.begin, si.count, XE, P, Q, ih2, bad, NB);
          break;
      }
      Ops<T>::check_launch();
    }
  }

  // Q = (M - K) P on free vertices, -(K P) on pinned ones (K with projected
  // blocks when pd)
  static void apply(xpbd_ctx c, const Dev<T>& D, const V4* XE, const D4* P, D4* Q, int* bad, const Work& w,
                    bool pd, hipStream_t st) {
    k_imp_mass<T><<<nblocks(c->V), kBlock, 0, st>>>((const V4*)c->XB, P, Q, c->V);
    Ops<T>::check_launch();
    if (pd) sets<IMP_APPLY_PD>(c, D, XE, P, Q, 0.0, bad, w, st);
    else sets<IMP_APPLY>(c, D, XE, P, Q, 0.0, bad, w, st);
  }

  // a . b (see k_imp_dot) into the device scalar *out, without the host
  static void dot_dev(xpbd_ctx c, const Work& w, const D4* a, const D4* b, const D4* diag, double* out,
                      hipStream_t st) {
    const unsigned nb = nblocks(c->V);
    k_imp_dot<<<nb, kBlock, 0, st>>>(a, b, diag, c->V, w.part);
    k_sum_parts<<<1, 1024, 0, st>>>(w.part, nb, out, 0);
    Ops<T>::check_launch();
  }

  static double dot(xpbd_ctx c, const Work& w, const D4* a, const D4* b, const D4* diag, hipStream_t st) {
    const unsigned nb = nblocks(c->V);
    k_imp_dot<<<nb, kBlock, 0, st>>>(a, b, diag, c->V, w.part);
    k_sum_parts<<<1, 1024, 0, st>>>(w.part, nb, w.sum, 0);
    Ops<T>::check_launch();
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, w.sum, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return v;
  }

  static void adjoint(xpbd_ctx c, const xpbd_params* p, const void* dLdx, const uint8_t* mask, xpbd_cg* cg,
                      const xpbd_grads* out, hipStream_t st) {
    const int V = c->V, F = c->fwd_frames, S = c->S;
    const double h = c->h, ih2 = 1.0 / (h * h);
    Ops<T>::gather_params(c, p, st);
    Dev<T> D = Ops<T>::dev(c, p->sphere);
    const bool pd = cg->pd_projection != 0;
    Work w = work(c, pd);
    HIPCHK(hipMemsetAsync(w.bad, 0, sizeof(int), st));
    Ops<T>::template fill<double>(c->dist_acc, 0.0, c->n_dist, st);
    Ops<T>::template fill<double>(c->bend_acc, 0.0, c->n_bend, st);
    if (out->f_ext) Ops<T>::template fill<T>((T*)out->f_ext, T(0), (size_t)F * 3 * V, st);
    k_adj_init<T><<<nblocks(V), kBlock, 0, st>>>((V4*)c->XB, (V4*)c->VB, (const T*)c->w, nullptr, V);
    Ops<T>::check_launch();
    const size_t vb = (size_t)V * sizeof(V4);
    int64_t total = 0;
    int most = 0;
    double worst = 0.0;
    for (int f = F - 1; f >= 0; --f) {
      if (dLdx && (!mask || mask[f])) {
        k_adj_inject<T><<<nblocks(V), kBlock, 0, st>>>((V4*)c->XB, (const T*)dLdx + (size_t)f * 3 * V, V);
        Ops<T>::check_launch();
      }
      const T* ff = p->f_ext ? (const T*)p->f_ext + (size_t)f * 3 * V : nullptr;
      T* fb = out->f_ext ? (T*)out->f_ext + (size_t)f * 3 * V : nullptr;
      Ops<T>::restore(c, f, st);
      for (int s = 0; s < S; ++s) {
        Ops<T>::substep(c, D, ff, -1, st);
        HIPCHK(hipMemcpyAsync((char*)w.XS + s * vb, c->X, vb, hipMemcpyDeviceToDevice, st));
      }
      for (int s = S - 1; s >= 0; --s) {
        const V4* XE = w.XS + (size_t)s * V;
        k_rev_velocity<T><<<nblocks(V), kBlock, 0, st>>>(D);
        Ops<T>::template fill<double>((double*)w.DG, 0.0, (size_t)4 * V, st);
        if (pd) {
          sets<IMP_BUILD>(c, D, XE, nullptr, nullptr, 0.0, w.bad, w, st);
          sets<IMP_DIAG_PD>(c, D, XE, nullptr, w.DG, 0.0, w.bad, w, st);
        } else {
          sets<IMP_DIAG>(c, D, XE, nullptr, w.DG, 0.0, w.bad, w, st);
        }
        k_imp_diag<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->XB, w.DG, V);
        if (s == S - 1 && f == F - 1) {
          int bad0 = 0;
          HIPCHK(hipMemcpyAsync(&bad0, w.bad, sizeof(int), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          if (bad0) fail(XPBD_ERR_INVALID, "implicit adjoint: an active constraint has zero compliance");
        }
        k_imp_rhs<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->XB, w.B, w.Y, w.R, V);
        Ops<T>::check_launch();
        const double bn = std::sqrt(dot(c, w, w.B, nullptr, nullptr, st));
        int it = 0;
        double rel = 0.0;
        if (bn > 0.0) {
          // preconditioned CG with its scalars on the device: batches of
          // iterations (8, doubling to 32) between the host's looks at the
          // state, the iterations after a stop leaving the solution as it is
          k_imp_dir<<<nblocks(V), kBlock, 0, st>>>(0.0, w.R, w.DG, w.P, V, 1);
          dot_dev(c, w, w.R, w.R, w.DG, w.cg + CG_RZ, st);
          k_cg_start<<<1, 1, 0, st>>>(w.cg, w.cgs);
          Ops<T>::check_launch();
          int state[2] = {CG_RUN, 0};
          for (int batch = 8; state[0] == CG_RUN; batch = std::min(2 * batch, 32)) {
            for (int b = 0; b < batch; ++b) {
              apply(c, D, XE, w.P, w.Q, w.bad, w, pd, st);
              dot_dev(c, w, w.P, w.Q, nullptr, w.cg + CG_PQ, st);
              k_cg_alpha<<<1, 1, 0, st>>>(w.cg, w.cgs);
              k_cg_axpy2<<<nblocks(V), kBlock, 0, st>>>(w.cg, w.cgs, w.P, w.Q, w.DG, w.Y, w.R, V);
              dot_dev(c, w, w.R, nullptr, nullptr, w.cg + CG_RR, st);
              k_cg_check<<<1, 1, 0, st>>>(w.cg, w.cgs, bn, cg->rel_tolerance, cg->max_iterations);
              dot_dev(c, w, w.R, w.R, w.DG, w.cg + CG_RZ2, st);
              k_cg_beta<<<1, 1, 0, st>>>(w.cg, w.cgs);
              k_cg_dir<<<nblocks(V), kBlock, 0, st>>>(w.cg, w.cgs, w.R, w.DG, w.P, V);
              Ops<T>::check_launch();
            }
            double sc[CG_NSLOT];
            HIPCHK(hipMemcpyAsync(state, w.cgs, sizeof(state), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(sc, w.cg, sizeof(sc), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            it = state[1];
            rel = sc[CG_REL];
            if (state[0] == CG_INDEFINITE)
              fail(XPBD_ERR_SOLVER,
                   "implicit adjoint: the system of frame %d, substep %d is not positive definite (p.Ap = %g)", f, s,
                   sc[CG_PQ]);
          }
        }
        total += it;
        most = std::max(most, it);
        worst = std::max(worst, rel);
        apply(c, D, XE, w.Y, w.Q, w.bad, w, pd, st);
        sets<IMP_GRAD>(c, D, XE, w.Y, nullptr, ih2, w.bad, w, st);
        k_imp_finish<T><<<nblocks(V), kBlock, 0, st>>>((V4*)c->XB, (V4*)c->VB, w.Y, w.Q, fb, h, V);
        Ops<T>::check_launch();
      }
    }
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) fail(XPBD_ERR_INVALID, "implicit adjoint: an active constraint has zero compliance");
    cg->total_iterations = total;
    cg->max_iterations_used = most;
    cg->worst_rel_residual = worst;
    if (out->x0) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->XB, (T*)out->x0, V);
    if (out->v0) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->VB, (T*)out->v0, V);
    if (out->dist_compliance && c->n_dist)
      k_scatter_alpha_grad<<<nblocks(c->n_dist), kBlock, 0, st>>>(c->dist_acc, c->dist_perm, out->dist_compliance,
                                                                  1.0, c->n_dist);
    if (out->bend_compliance && c->n_bend)
      k_scatter_alpha_grad<<<nblocks(c->n_bend), kBlock, 0, st>>>(c->bend_acc, c->bend_perm, out->bend_compliance,
                                                                  1.0, c->n_bend);
    Ops<T>::check_launch();
  }
};

}  // namespace

extern "C" {

xpbd_status xpbd_adjoint_implicit(xpbd_ctx c, const xpbd_params* p, const void* dLdx_frames,
                                  const uint8_t* frame_mask, xpbd_cg* cg, const xpbd_grads* out, void* stream) {
  if (!c) return XPBD_ERR_INVALID;
  return guarded(c, [&] {
    if (c->in_pack) fail(XPBD_ERR_STATE, "implicit adjoint: the context is serving a job of a pack");
    if (!p || !out || !cg) fail(XPBD_ERR_INVALID, "implicit adjoint: null argument");
    if (cg->max_iterations < 1 || !(cg->rel_tolerance > 0.0))
      fail(XPBD_ERR_INVALID, "implicit adjoint: max_iterations >= 1 and rel_tolerance > 0 required");
    if (out->tet_E || out->sphere || out->tet_mu || out->tet_lambda || out->tri_coef || out->body_x)
      fail(XPBD_ERR_INVALID,
           "implicit adjoint: tet, membrane and sphere parameter gradients are not produced (pass NULL)");
    if (c->n_tri || c->n_bc)
      fail(XPBD_ERR_INVALID, "implicit adjoint: membrane triangles and body contacts are not supported");
    if (!c->have_forward) fail(XPBD_ERR_STATE, "implicit adjoint: no preceding forward on this context");
    const xpbd_params& q = c->fwd_params;
    if (q.dist_compliance != p->dist_compliance || q.bend_compliance != p->bend_compliance ||
        q.tet_E != p->tet_E || q.f_ext != p->f_ext || std::memcmp(q.sphere, p->sphere, sizeof q.sphere) != 0 ||
        q.tet_mu != p->tet_mu || q.tet_lambda != p->tet_lambda || q.tri_coef != p->tri_coef ||
        q.body_x != p->body_x)
      fail(XPBD_ERR_STATE, "implicit adjoint: parameters differ from the preceding forward");
    ensure_adjoint_buffers(c, 0);
    hipStream_t st = (hipStream_t)stream;
    if (c->dtype == XPBD_F32) ImpOps<float>::adjoint(c, p, dLdx_frames, frame_mask, cg, out, st);
    else ImpOps<double>::adjoint(c, p, dLdx_frames, frame_mask, cg, out, st);
  });
}

}  // extern "C"
