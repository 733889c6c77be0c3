// Host side of packs (the "packs" part of include/xpbd.h): job admission,
// the round plan that merges the same step of every job into one launch,
// HIP graph capture of a round, and each job's phase changes (forward ->
// goal and adjoint -> done).  Included once, at the end of xpbd.hip.
#pragma once

struct xpbd_pack_s {
  std::string err;
  xpbd_dtype dtype = XPBD_F32;
  bool graphs = false;
  int block = kBlock;   // workgroup size of the set and vertex launches
  int S = -1, K = -1;

  struct Job {
    int64_t id = 0;
    xpbd_ctx c = nullptr;
    xpbd_job j{};
    std::vector<uint8_t> mask;   // host copy, for the goal
    int phase = 0;               // 0 forward rollout, 1 adjoint
    int f = 0;                   // frame the next round works on
    int mode = 0;                // adjoint record: 3 whole rollout, 1 one frame; 0 no adjoint
  };
  std::vector<Job> jobs;
  std::vector<int64_t> done;     // finished, not yet reported
  int64_t next_id = 1;
  bool dirty = true;             // jobs or phases changed since the plan was built

  enum { L_VERT, L_FWD, L_REV, L_SPHERE, L_ADVANCE };
  struct Launch {
    int kind;
    int op;          // vertex op, or constraint type (-1 = mixed)
    bool first, last;
    int slot_it;     // substep * K + iteration
    unsigned grid;
    size_t seg;      // first segment in the table
    int nseg;
  };
  // Two plan slots used in turn, so that building a new plan never waits for
  // the rounds of the current one: a slot is reused only after the last
  // round that read its tables (an event recorded after every round).
  struct Slot {
    std::vector<Launch> plan;
    int n_members = 0;
    void* dmem = nullptr; size_t dmem_cap = 0;   // member table (device)
    void* dseg = nullptr; size_t dseg_cap = 0;   // segment tables (device)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;                   // after the slot's last round
    bool pending = false;
    void drop_graph() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
  };
  Slot slot[2];
  int cur = -1;

  hipStream_t cap_stream = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
  // admission work (parameter checks, initial state) runs on its own stream
  // so that adding a job never waits for the pack's rounds
  hipStream_t adm_stream = nullptr;
  hipEvent_t adm_event = nullptr;
  bool adm_pending = false;
  xpbd_pack_stats stats{};

  ~xpbd_pack_s() {
    if (used) (void)hipStreamSynchronize(last_stream);
    for (Slot& s : slot) {
      s.drop_graph();
      if (s.dmem) (void)hipFree(s.dmem);
      if (s.dseg) (void)hipFree(s.dseg);
      if (s.done) (void)hipEventDestroy(s.done);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (adm_stream) {
      (void)hipStreamSynchronize(adm_stream);
      (void)hipStreamDestroy(adm_stream);
    }
    if (adm_event) (void)hipEventDestroy(adm_event);
    for (auto& J : jobs) J.c->in_pack = false;
  }
};

namespace {

void pack_grow(void*& p, size_t& cap, size_t bytes) {
  if (bytes <= cap) return;
  if (p) HIPCHK(hipFree(p));
  p = nullptr;
  cap = 0;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    fail(XPBD_ERR_OOM, "pack tables: hipMalloc(%zu) failed", bytes);
  }
  cap = bytes;
}

template <class T> struct PackOps {
  using V4 = Vec4<T>;
  using Job = xpbd_pack_s::Job;
  using Launch = xpbd_pack_s::Launch;

  static void check_launch() { Ops<T>::check_launch(); }

  // ---------------------------------------------------------------- admission
  static void add(xpbd_pack pk, xpbd_ctx c, const xpbd_job* j, hipStream_t st, int64_t* id) {
    const int F = j->n_frames;
    if (!j->x0 || !j->v0 || F < 1) fail(XPBD_ERR_INVALID, "pack add: null x0 / v0 or n_frames < 1");
    if (c->n_tet && !j->params.tet_E && !(j->params.tet_mu && j->params.tet_lambda))
      fail(XPBD_ERR_INVALID, "pack add: tet_E, or tet_mu and tet_lambda, required");
    if (c->n_tri && !j->params.tri_coef) fail(XPBD_ERR_INVALID, "pack add: tri_coef required");
    if (c->n_bc) fail(XPBD_ERR_INVALID, "pack add: body-contact meshes are not packed");
    if (c->record_kind) fail(XPBD_ERR_INVALID, "pack add: contexts with snapshot records are not packed");
    const bool adj = j->targets != nullptr;
    if (adj && !j->x_frames) fail(XPBD_ERR_INVALID, "pack add: a job with an adjoint needs x_frames");
    c->have_forward = false;
    c->fwd_recorded = false;
    // the context's previous job (in any pack) must be finished on the
    // device before its buffers are reused
    if (c->pack_event) HIPCHK(hipEventSynchronize(c->pack_event));
    if (!pk->adm_stream) {
      HIPCHK(hipStreamCreateWithFlags(&pk->adm_stream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&pk->adm_event, hipEventDisableTiming));
    }
    (void)st;
    st = pk->adm_stream;
    Ops<T>::gather_params(c, &j->params, st);
    ensure_checkpoints(c, F);
    Job J;
    J.c = c;
    J.j = *j;
    if (adj) {
      const size_t frame = (size_t)c->S * c->K * c->iter_tape_bytes;
      const int opt = c->tape_mode_opt;
      if (opt == 2) fail(XPBD_ERR_INVALID, "pack add: tape_mode 2 (per-substep recomputation) is not available in packs");
      if ((opt == 0 || opt == 3) && fits_on_device(c, (size_t)F * frame)) {
        J.mode = 3;
        ensure_adjoint_buffers(c, F * c->S);
      } else if (opt == 3) {
        fail(XPBD_ERR_OOM, "pack add: the record of the whole rollout (%zu bytes) does not fit", (size_t)F * frame);
      } else if (fits_on_device(c, frame)) {
        J.mode = 1;
        ensure_adjoint_buffers(c, c->S);
      } else {
        fail(XPBD_ERR_OOM, "pack add: the record of one frame (%zu bytes) does not fit", frame);
      }
      J.mask.assign(F, 1);
      if (j->frame_mask)
        for (int f = 0; f < F; ++f) J.mask[f] = j->frame_mask[f] ? 1 : 0;
      if (c->pack_mask_cap < F) {
        void* pm = c->pack_mask;
        c->release(pm);
        c->pack_mask = nullptr;
        c->pack_mask_cap = 0;
        c->pack_mask = (uint8_t*)c->alloc((size_t)F);
        c->pack_mask_cap = F;
      }
      HIPCHK(hipMemcpy(c->pack_mask, J.mask.data(), (size_t)F, hipMemcpyHostToDevice));
      if (j->loss) Ops<T>::ensure_parts(c, F);
    }
    k_pack<T><<<nblocks(c->V), kBlock, 0, st>>>((const T*)j->x0, (const T*)j->v0, (const T*)c->w, (V4*)c->X,
                                                 (V4*)c->Vv, c->V);
    check_launch();
    HIPCHK(hipEventRecord(pk->adm_event, st));
    pk->adm_pending = true;
    if (!c->pack_event) HIPCHK(hipEventCreateWithFlags(&c->pack_event, hipEventDisableTiming));
    J.id = pk->next_id++;
    pk->jobs.push_back(J);
    c->in_pack = true;
    pk->dirty = true;
    *id = J.id;
  }

  // ---------------------------------------------------------------- round plan
  static bool fwd_kind(const Job& J) { return J.phase == 0 || J.mode == 1; }

  static void build_plan(xpbd_pack pk, hipStream_t st) {
    const int next = (pk->cur + 1) % 2;
    xpbd_pack_s::Slot& SL = pk->slot[next];
    if (SL.pending) HIPCHK(hipEventSynchronize(SL.done));   // its last round has finished
    SL.pending = false;
    SL.drop_graph();
    if (!SL.done) HIPCHK(hipEventCreateWithFlags(&SL.done, hipEventDisableTiming));
    const int M = (int)pk->jobs.size();
    const int S = pk->S, K = pk->K;
    std::vector<PackMember<T>> mem(M);
    for (int m = 0; m < M; ++m) {
      const Job& J = pk->jobs[m];
      xpbd_ctx c = J.c;
      PackMember<T>& P = mem[m];
      P.D = Ops<T>::dev(c, J.j.params.sphere);
      P.f = J.f;
      P.dir = J.phase == 0 ? 1 : -1;
      P.tape = (char*)c->tape;
      P.iter_tape = (long long)c->iter_tape_bytes;
      P.frame_tape = J.mode == 3 ? (long long)S * K * (long long)c->iter_tape_bytes : 0;
      P.fext = (const T*)J.j.params.f_ext;
      P.fbar = J.phase == 1 ? (T*)J.j.grads.f_ext : nullptr;
      P.xf = (T*)J.j.x_frames;
      P.tgt = (const T*)J.j.targets;
      P.mask = c->pack_mask;
      P.ckX = (V4*)c->ckX;
      P.ckV = (V4*)c->ckV;
      P.dsph = J.phase == 1 ? J.j.grads.sphere : nullptr;
    }
    std::vector<PackSeg> seg;
    std::vector<Launch> plan;
    auto vert = [&](int op, auto pick) {
      size_t s0 = seg.size();
      int b = 0;
      for (int m = 0; m < M; ++m)
        if (pick(pk->jobs[m])) {
          PackSeg g{m, 0, 0, pk->jobs[m].c->V, b, 0, 0};
          seg.push_back(g);
          b += (int)nblocks(g.count, pk->block);
        }
      if (b) plan.push_back({xpbd_pack_s::L_VERT, op, false, false, 0, (unsigned)b, s0, (int)(seg.size() - s0)});
    };
    auto sets = [&](bool rev, int k, bool first, bool last, int slot_it, auto pick) {
      size_t s0 = seg.size();
      int b = 0, ty = -2;
      for (int m = 0; m < M; ++m) {
        const Job& J = pk->jobs[m];
        if (!pick(J) || k >= (int)J.c->sets.size()) continue;
        const SetInfo& si = J.c->sets[k];
        if (si.count == 0) continue;
        int tape = rev ? 1 : ((J.phase == 0 && J.mode == 3) || J.phase == 1) ? 1 : 0;
        seg.push_back(PackSeg{m, si.type, si.begin, si.count, b, tape, (long long)si.tape_off});
        b += (int)nblocks(si.count, pk->block);
        ty = ty == -2 ? si.type : (ty == si.type ? ty : -1);
      }
      if (b)
        plan.push_back({rev ? xpbd_pack_s::L_REV : xpbd_pack_s::L_FWD, ty, first, last, slot_it, (unsigned)b, s0,
                        (int)(seg.size() - s0)});
    };
    int max_fwd = 0, max_rev = 0, max_contact = 0;
    bool any_fwd_phase = false, any_restore = false, any_unpack = false, any_rev = false, any_fwd = false;
    for (const Job& J : pk->jobs) {
      int ns = (int)J.c->sets.size(), nc = 0;
      for (const SetInfo& si : J.c->sets) nc += si.type == XPBD_CONTACT && si.count > 0;
      if (fwd_kind(J)) { any_fwd = true; max_fwd = std::max(max_fwd, ns); }
      if (J.phase == 0) { any_fwd_phase = true; any_unpack |= J.j.x_frames != nullptr; }
      if (J.phase == 1) {
        any_rev = true;
        max_rev = std::max(max_rev, ns);
        any_restore |= J.mode == 1;
        if (J.j.grads.sphere) max_contact = std::max(max_contact, nc);
      }
    }
    auto is_fwd_phase = [](const Job& J) { return J.phase == 0; };
    auto is_rev = [](const Job& J) { return J.phase == 1; };
    if (any_fwd_phase) vert(PV_CHECKPOINT, is_fwd_phase);
    if (any_restore) vert(PV_RESTORE, [](const Job& J) { return J.phase == 1 && J.mode == 1; });
    if (any_fwd) {
      for (int s = 0; s < S; ++s) {
        vert(PV_PREDICT, fwd_kind);
        for (int it = 0; it < K; ++it)
          for (int k = 0; k < max_fwd; ++k) sets(false, k, it == 0, false, s * K + it, fwd_kind);
        vert(PV_VELOCITY, fwd_kind);
      }
    }
    if (any_unpack) vert(PV_UNPACK, [](const Job& J) { return J.phase == 0 && J.j.x_frames != nullptr; });
    if (any_rev) {
      vert(PV_INJECT, is_rev);
      for (int s = S - 1; s >= 0; --s) {
        vert(PV_REV_VELOCITY, is_rev);
        for (int it = K - 1; it >= 0; --it)
          for (int k = max_rev - 1; k >= 0; --k) sets(true, k, it == K - 1, it == 0, s * K + it, is_rev);
        if (K > 0)
          for (int q = 0; q < max_contact; ++q) {
            // the q-th non-empty contact set of each job that wants the sphere gradient
            size_t s0 = seg.size();
            for (int m = 0; m < M; ++m) {
              const Job& J = pk->jobs[m];
              if (J.phase != 1 || !J.j.grads.sphere) continue;
              int n = 0;
              for (const SetInfo& si : J.c->sets)
                if (si.type == XPBD_CONTACT && si.count > 0 && n++ == q)
                  seg.push_back(PackSeg{m, XPBD_CONTACT, si.begin, si.count, (int)(seg.size() - s0), 0, 0});
            }
            int ns = (int)(seg.size() - s0);
            if (ns) plan.push_back({xpbd_pack_s::L_SPHERE, 0, false, false, 0, (unsigned)ns, s0, ns});
          }
        vert(PV_REV_PREDICT, is_rev);
      }
    }
    if (M) plan.push_back({xpbd_pack_s::L_ADVANCE, 0, false, false, 0, nblocks(M), 0, 0});
    pack_grow(SL.dmem, SL.dmem_cap, std::max<size_t>(1, (size_t)M) * sizeof(PackMember<T>));
    pack_grow(SL.dseg, SL.dseg_cap, std::max<size_t>(1, seg.size()) * sizeof(PackSeg));
    // host-synchronous copies: complete before any later launch reads them,
    // and nothing in flight reads this slot any more
    if (M) HIPCHK(hipMemcpy(SL.dmem, mem.data(), (size_t)M * sizeof(PackMember<T>), hipMemcpyHostToDevice));
    if (!seg.empty()) HIPCHK(hipMemcpy(SL.dseg, seg.data(), seg.size() * sizeof(PackSeg), hipMemcpyHostToDevice));
    (void)st;
    SL.plan.swap(plan);
    SL.n_members = M;
    pk->cur = next;
    pk->stats.last_round_launches = (int32_t)SL.plan.size();
    pk->dirty = false;
  }

  // ---------------------------------------------------------------- launches
  template <int TY>
  static void fwd(const Launch& L, const PackMember<T>* mem, const PackSeg* sg, int blk, hipStream_t st) {
    if (L.first) k_pack_fwd<T, TY, true><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg, L.slot_it);
    else k_pack_fwd<T, TY, false><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg, L.slot_it);
  }
  template <int TY>
  static void rev(const Launch& L, const PackMember<T>* mem, const PackSeg* sg, int blk, hipStream_t st) {
    if (L.first) {
      if (L.last) k_pack_rev<T, TY, true, true><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg, L.slot_it);
      else k_pack_rev<T, TY, true, false><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg, L.slot_it);
    } else {
      if (L.last) k_pack_rev<T, TY, false, true><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg, L.slot_it);
      else k_pack_rev<T, TY, false, false><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg, L.slot_it);
    }
  }

  static void launch_plan(xpbd_pack pk, hipStream_t st) {
    const xpbd_pack_s::Slot& SL = pk->slot[pk->cur];
    PackMember<T>* mem = (PackMember<T>*)SL.dmem;
    const PackSeg* seg0 = (const PackSeg*)SL.dseg;
    const int n_members = SL.n_members;
    const int blk = pk->block;
    for (const Launch& L : SL.plan) {
      const PackSeg* sg = seg0 + L.seg;
      switch (L.kind) {
        case xpbd_pack_s::L_VERT:
          switch (L.op) {
            case PV_CHECKPOINT: k_pack_vert<T, PV_CHECKPOINT><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
            case PV_RESTORE: k_pack_vert<T, PV_RESTORE><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
            case PV_PREDICT: k_pack_vert<T, PV_PREDICT><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
            case PV_VELOCITY: k_pack_vert<T, PV_VELOCITY><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
            case PV_UNPACK: k_pack_vert<T, PV_UNPACK><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
            case PV_INJECT: k_pack_vert<T, PV_INJECT><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
            case PV_REV_VELOCITY:
              k_pack_vert<T, PV_REV_VELOCITY><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg);
              break;
            default: k_pack_vert<T, PV_REV_PREDICT><<<L.grid, blk, 0, st>>>(mem, sg, L.nseg); break;
          }
          break;
        case xpbd_pack_s::L_FWD:
          switch (L.op) {
            case 0: fwd<0>(L, mem, sg, blk, st); break;
            case 1: fwd<1>(L, mem, sg, blk, st); break;
            case 2: fwd<2>(L, mem, sg, blk, st); break;
            case 3: fwd<3>(L, mem, sg, blk, st); break;
            case 4: fwd<4>(L, mem, sg, blk, st); break;
            default: fwd<-1>(L, mem, sg, blk, st); break;
          }
          break;
        case xpbd_pack_s::L_REV:
          switch (L.op) {
            case 0: rev<0>(L, mem, sg, blk, st); break;
            case 1: rev<1>(L, mem, sg, blk, st); break;
            case 2: rev<2>(L, mem, sg, blk, st); break;
            case 3: rev<3>(L, mem, sg, blk, st); break;
            case 4: rev<4>(L, mem, sg, blk, st); break;
            default: rev<-1>(L, mem, sg, blk, st); break;
          }
          break;
        case xpbd_pack_s::L_SPHERE: k_pack_sphere<T><<<L.grid, kBlock, 0, st>>>(mem, sg); break;
        default: k_pack_advance<T><<<L.grid, kBlock, 0, st>>>(mem, n_members); break;
      }
      check_launch();
    }
  }

  static void capture(xpbd_pack pk) {
    xpbd_pack_s::Slot& SL = pk->slot[pk->cur];
    if (!pk->cap_stream) HIPCHK(hipStreamCreateWithFlags(&pk->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(pk->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      launch_plan(pk, pk->cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(pk->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(pk->cap_stream, &SL.graph));
    HIPCHK(hipGraphInstantiate(&SL.exec, SL.graph, nullptr, nullptr, 0));
    pk->stats.graph_captures += 1;
  }

  // ---------------------------------------------------------------- phase changes
  static void finish_job(xpbd_pack pk, Job& J, hipStream_t st) {
    HIPCHK(hipEventRecord(J.c->pack_event, st));
    J.c->in_pack = false;
    pk->done.push_back(J.id);
  }

  static void after_round(xpbd_pack pk, hipStream_t st) {
    std::vector<Job> keep;
    keep.reserve(pk->jobs.size());
    for (Job& J : pk->jobs) {
      xpbd_ctx c = J.c;
      const int F = J.j.n_frames, V = c->V;
      J.f += J.phase == 0 ? 1 : -1;
      if (J.phase == 0 && J.f == F) {
        if (J.j.x_final) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->X, (T*)J.j.x_final, V);
        if (J.j.v_final) k_unpack<T><<<nblocks(V), kBlock, 0, st>>>((const V4*)c->Vv, (T*)J.j.v_final, V);
        check_launch();
        pk->dirty = true;
        if (!J.j.targets) {
          finish_job(pk, J, st);
          continue;
        }
        if (J.j.loss) Ops<T>::goal(c, J.j.x_frames, J.j.targets, J.mask.data(), nullptr, F, J.j.loss, nullptr, st);
        Ops<T>::begin_adjoint(c, F, J.j.dLdv_final, &J.j.grads, st);
        J.phase = 1;
        J.f = F - 1;
      } else if (J.phase == 1 && J.f < 0) {
        Ops<T>::finish_adjoint(c, &J.j.params, &J.j.grads, st);
        pk->dirty = true;
        finish_job(pk, J, st);
        continue;
      }
      keep.push_back(J);
    }
    pk->jobs.swap(keep);
  }

  static void run(xpbd_pack pk, int max_rounds, hipStream_t st) {
    for (int r = 0; r < max_rounds && !pk->jobs.empty(); ++r) {
      if (pk->adm_pending) {
        HIPCHK(hipStreamWaitEvent(st, pk->adm_event, 0));
        pk->adm_pending = false;
      }
      if (pk->dirty) build_plan(pk, st);
      xpbd_pack_s::Slot& SL = pk->slot[pk->cur];
      if (pk->graphs) {
        if (!SL.exec) capture(pk);
        HIPCHK(hipGraphLaunch(SL.exec, st));
        pk->stats.graph_launches += 1;
      } else {
        launch_plan(pk, st);
        pk->stats.launches += (int64_t)SL.plan.size();
      }
      HIPCHK(hipEventRecord(SL.done, st));
      SL.pending = true;
      pk->used = true;
      pk->last_stream = st;
      pk->stats.rounds += 1;
      size_t before = pk->done.size();
      after_round(pk, st);
      if (pk->done.size() > before) break;
    }
  }
};

template <class F> xpbd_status pack_guarded(xpbd_pack pk, F&& fn) {
  try {
    fn();
    pk->err.clear();
    return XPBD_OK;
  } catch (const Fail& f) {
    pk->err = f.msg;
    return f.st;
  } catch (const std::bad_alloc&) {
    pk->err = "host allocation failed";
    return XPBD_ERR_OOM;
  } catch (...) {
    pk->err = "unexpected exception";
    return XPBD_ERR_HIP;
  }
}

}  // namespace

extern "C" {

xpbd_status xpbd_pack_create(xpbd_dtype dtype, int32_t flags, int32_t block_size, xpbd_pack* out) {
  if (!out) return XPBD_ERR_INVALID;
  *out = nullptr;
  if ((dtype != XPBD_F32 && dtype != XPBD_F64) || (flags & ~XPBD_PACK_GRAPHS)) return XPBD_ERR_INVALID;
  if (block_size != 0 && block_size != 64 && block_size != 128 && block_size != 256) return XPBD_ERR_INVALID;
  xpbd_pack pk = nullptr;
  try {
    pk = new xpbd_pack_s();
  } catch (...) {
    return XPBD_ERR_OOM;
  }
  pk->dtype = dtype;
  pk->graphs = (flags & XPBD_PACK_GRAPHS) != 0;
  pk->block = block_size ? block_size : kBlock;
  *out = pk;
  return XPBD_OK;
}

xpbd_status xpbd_pack_destroy(xpbd_pack pk) {
  if (!pk) return XPBD_ERR_INVALID;
  delete pk;
  return XPBD_OK;
}

xpbd_status xpbd_pack_add(xpbd_pack pk, xpbd_ctx c, const xpbd_job* job, void* stream, int64_t* job_id) {
  if (!pk) return XPBD_ERR_INVALID;
  return pack_guarded(pk, [&] {
    if (!c || !job || !job_id) fail(XPBD_ERR_INVALID, "pack add: null argument");
    if (c->in_pack) fail(XPBD_ERR_INVALID, "pack add: the context is already serving a job");
    if (c->dtype != pk->dtype) fail(XPBD_ERR_INVALID, "pack add: context dtype differs from the pack's");
    if (pk->S >= 0 && (c->S != pk->S || c->K != pk->K))
      fail(XPBD_ERR_INVALID, "pack add: substeps / iterations (%d, %d) differ from the pack's (%d, %d)", c->S, c->K,
           pk->S, pk->K);
    hipStream_t st = (hipStream_t)stream;
    try {
      if (c->dtype == XPBD_F32) PackOps<float>::add(pk, c, job, st, job_id);
      else PackOps<double>::add(pk, c, job, st, job_id);
    } catch (const Fail& f) {
      c->err = f.msg;
      throw;
    }
    pk->S = c->S;
    pk->K = c->K;
  });
}

xpbd_status xpbd_pack_run(xpbd_pack pk, int32_t max_rounds, void* stream, int64_t* done_ids, int32_t cap,
                          int32_t* n_done) {
  if (!pk) return XPBD_ERR_INVALID;
  return pack_guarded(pk, [&] {
    if (max_rounds < 0 || cap < 0 || (cap > 0 && !done_ids)) fail(XPBD_ERR_INVALID, "pack run: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    if (pk->used && st != pk->last_stream) HIPCHK(hipStreamSynchronize(pk->last_stream));
    if (pk->dtype == XPBD_F32) PackOps<float>::run(pk, max_rounds, st);
    else PackOps<double>::run(pk, max_rounds, st);
    int n = (int)std::min<size_t>((size_t)cap, pk->done.size());
    for (int i = 0; i < n; ++i) done_ids[i] = pk->done[i];
    pk->done.erase(pk->done.begin(), pk->done.begin() + n);
    if (n_done) *n_done = n;
  });
}

xpbd_status xpbd_pack_get_stats(xpbd_pack pk, xpbd_pack_stats* stats) {
  if (!pk || !stats) return XPBD_ERR_INVALID;
  *stats = pk->stats;
  stats->active_jobs = (int32_t)pk->jobs.size();
  return XPBD_OK;
}

const char* xpbd_pack_last_error(xpbd_pack pk) { return pk ? pk->err.c_str() : ""; }

}  // extern "C"
