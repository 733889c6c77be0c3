// Packed launches: one launch serves the same step of many independent
// contexts (meshes of any size and constraint mix).  A launch's blocks are
// split into segments, one per (context, set) or (context, vertex range);
// each block finds its segment by binary search over the segments' first
// block, then runs exactly the per-item code of the one-context kernels
// (one item per thread; the workgroup size, 64, 128 or 256, is the pack's), so
// every context's results are bitwise those of running it alone.
//
// Each context's frame index lives in device memory and is advanced by the
// last launch of a round, so a round's launch sequence does not change from
// frame to frame and can be captured once in a HIP graph and replayed.
#pragma once

#include "xpbd_kernels.hpp"

namespace xpbd {

struct PackSeg {
  int member;          // row of the member table
  int type;            // constraint type (set launches)
  int begin;           // first internal record of the set (set launches)
  int count;           // items (set launches) or vertices (vertex launches)
  int block0;          // first block of the segment inside its launch
  int tape;            // forward: 1 = write the adjoint's record of this set
  long long tape_off;  // byte offset of the set's record inside one iteration
};

template <class T> struct PackMember {
  Dev<T> D;
  int f;                     // frame being worked on; advanced by k_pack_advance
  int dir;                   // +1 forward rollout, -1 adjoint
  char* tape;                // record base
  long long frame_tape;      // record bytes per frame (whole-rollout record), 0 = one frame kept
  long long iter_tape;       // record bytes per iteration
  const T* fext;             // [F][3V] external forces or null
  T* fbar;                   // [F][3V] force adjoints or null
  T* xf;                     // [F][3V] frame outputs or null
  const T* tgt;              // [F][3V] goal targets (adjoint)
  const unsigned char* mask; // [F] goal frames (adjoint)
  Vec4<T>* ckX;              // [F][V] checkpoints
  Vec4<T>* ckV;
  double* dsph;              // [4] sphere gradient or null
};

enum PackVertOp {
  PV_CHECKPOINT = 0,  // ck[f] = (x, v)
  PV_RESTORE,         // (x, v) = ck[f]
  PV_PREDICT,
  PV_VELOCITY,
  PV_UNPACK,          // x_frames[f] = x
  PV_INJECT,          // xbar += x(f) - x*(f) on goal frames
  PV_REV_VELOCITY,
  PV_REV_PREDICT
};

__device__ __forceinline__ int pack_find(const PackSeg* __restrict__ seg, int nseg, int b) {
  int lo = 0, hi = nseg;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (seg[mid].block0 <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <class T>
__device__ __forceinline__ char* pack_tape(const PackMember<T>& M, const PackSeg& S, int slot_it) {
  return M.tape + (long long)M.f * M.frame_tape + (long long)slot_it * M.iter_tape + S.tape_off;
}

// TY >= 0: every segment has that constraint type; TY < 0: per-segment type
template <class T, int TY, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_pack_fwd(const PackMember<T>* __restrict__ mem,
                                                     const PackSeg* __restrict__ seg, int nseg, int slot_it) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const PackSeg& S = seg[pack_find(seg, nseg, b)];
  const int t = (b - S.block0) * (int)blockDim.x + threadIdx.x;
  if (t >= S.count) return;
  const PackMember<T>& M = mem[S.member];
  const int ty = TY >= 0 ? TY : S.type;
  if (S.tape) {
    Vec4<T>* tp = reinterpret_cast<Vec4<T>*>(pack_tape(M, S, slot_it));
    switch (ty) {
      case 0: dist_item<T, FIRST, true>(M.D, S.begin, S.count, t, tp); break;
      case 1: bend_item<T, FIRST, true>(M.D, S.begin, S.count, t, tp); break;
      case 2: tet_item<T, FIRST, true>(M.D, S.begin, S.count, t, tp); break;
      case 4: tri_item<T, FIRST, true>(M.D, S.begin, S.count, t, tp); break;
      default: contact_item<T, FIRST, true>(M.D, S.begin, S.count, t, tp); break;
    }
  } else {
    switch (ty) {
      case 0: dist_item<T, FIRST, false>(M.D, S.begin, S.count, t, nullptr); break;
      case 1: bend_item<T, FIRST, false>(M.D, S.begin, S.count, t, nullptr); break;
      case 2: tet_item<T, FIRST, false>(M.D, S.begin, S.count, t, nullptr); break;
      case 4: tri_item<T, FIRST, false>(M.D, S.begin, S.count, t, nullptr); break;
      default: contact_item<T, FIRST, false>(M.D, S.begin, S.count, t, nullptr); break;
    }
  }
}

template <class T, int TY, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void k_pack_rev(const PackMember<T>* __restrict__ mem,
                                                     const PackSeg* __restrict__ seg, int nseg, int slot_it) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const PackSeg& S = seg[pack_find(seg, nseg, b)];
  const int t = (b - S.block0) * (int)blockDim.x + threadIdx.x;
  if (t >= S.count) return;
  const PackMember<T>& M = mem[S.member];
  const Vec4<T>* tp = reinterpret_cast<const Vec4<T>*>(pack_tape(M, S, slot_it));
  switch (TY >= 0 ? TY : S.type) {
    case 0: dist_rev_item<T, FIRST, LAST>(M.D, S.begin, S.count, t, tp); break;
    case 1: bend_rev_item<T, FIRST, LAST>(M.D, S.begin, S.count, t, tp); break;
    case 2: tet_rev_item<T, FIRST, LAST>(M.D, S.begin, S.count, t, tp); break;
    case 4: tri_rev_item<T, FIRST, LAST>(M.D, S.begin, S.count, t, tp); break;
    default: contact_rev_item<T, FIRST, LAST>(M.D, S.begin, S.count, t, tp); break;
  }
}

template <class T, int OP>
__global__ __launch_bounds__(kBlock) void k_pack_vert(const PackMember<T>* __restrict__ mem,
                                                      const PackSeg* __restrict__ seg, int nseg) {
  const int b = blockIdx.x;
  const PackSeg& S = seg[pack_find(seg, nseg, b)];
  const int k = (b - S.block0) * (int)blockDim.x + threadIdx.x;
  if (k >= S.count) return;
  const PackMember<T>& M = mem[S.member];
  const size_t V = (size_t)M.D.V, f = (size_t)M.f;
  switch (OP) {
    case PV_CHECKPOINT:
      M.ckX[f * V + k] = M.D.X[k];
      M.ckV[f * V + k] = M.D.Vv[k];
      break;
    case PV_RESTORE:
      M.D.X[k] = M.ckX[f * V + k];
      M.D.Vv[k] = M.ckV[f * V + k];
      break;
    case PV_PREDICT: predict_item(M.D, k, M.fext ? M.fext + f * 3 * V : nullptr); break;
    case PV_VELOCITY: velocity_item(M.D, k); break;
    case PV_UNPACK: {
      Vec4<T> p = M.D.X[k];
      T* o = M.xf + f * 3 * V + 3 * (size_t)k;
      o[0] = p.x; o[1] = p.y; o[2] = p.z;
      break;
    }
    case PV_INJECT:
      if (M.mask[f]) {
        const T* x = M.xf + f * 3 * V + 3 * (size_t)k;
        const T* g = M.tgt + f * 3 * V + 3 * (size_t)k;
        Vec4<T> p = M.D.XB[k];
        p.x += (T)(x[0] - g[0]); p.y += (T)(x[1] - g[1]); p.z += (T)(x[2] - g[2]);
        M.D.XB[k] = p;
      }
      break;
    case PV_REV_VELOCITY: rev_velocity_item(M.D, k); break;
    case PV_REV_PREDICT: rev_predict_item(M.D, k, M.fbar ? M.fbar + f * 3 * V : nullptr); break;
    default: break;
  }
}

// one block per segment: the sphere gradient of one contact set of one member
template <class T>
__global__ __launch_bounds__(kBlock) void k_pack_sphere(const PackMember<T>* __restrict__ mem,
                                                        const PackSeg* __restrict__ seg) {
  __shared__ double sh[4][kBlock];
  const PackSeg& S = seg[blockIdx.x];
  const PackMember<T>& M = mem[S.member];
  sphere_reduce_block<T, kBlock>(M.D.c_sacc, M.D.c_order, S.begin, S.count, M.dsph, sh);
}

// end of a round: every member moves to its next frame
template <class T>
__global__ __launch_bounds__(kBlock) void k_pack_advance(PackMember<T>* __restrict__ mem, int n) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) mem[i].f += mem[i].dir;
}

}  // namespace xpbd
