// Batches of independent systems: one launch per stage for all systems, FFTs
// batched per grid size, lockstep GMRES with per-system Krylov spaces, and a
// HIP graph of the preconditioner + saddle-operator sequence.
#include "ctx.h"

namespace fbim {
namespace {

template <class T>
T *carve(char *base, size_t &off, size_t n) {
  off = (off + 255) & ~(size_t)255;
  T *p = reinterpret_cast<T *>(base + off);
  off += n * sizeof(T);
  return p;
}

// FFT size class: systems sharing the grid size M transform together
struct SizeClass {
  int M = 0;
  std::vector<int> sys;  // engine system indices
  rocfft_plan fwd = nullptr, inv = nullptr, fwd32 = nullptr, inv32 = nullptr;
  double *grid = nullptr, *spec = nullptr;
  float *grid32 = nullptr, *spec32 = nullptr;
};

// Device job tables of one list of systems (the systems of one batched launch set).
struct Tables {
  int S = 0;
  std::vector<int> list;  // engine system indices, in table order
  GatherJob *gcell[2], *gtile[2];  // [0] FP64, [1] FP32 destinations
  PairJob *pair[2];
  AlpertJob *alp;
  SpreadJob *spr[2];
  MultJob *mul[2];
  InterpJob *itp[2];
  RigidJob *rig;
  PrecondJob *pre;
  BatchGrid bg_nodes{}, bg_pair{}, bg_tiles{}, bg_spec{}, bg_bodies4{}, bg_prec{};
  size_t prec_lds = 0;
  int prec_mfma = 0;  // row blocks per wave when every system takes the matrix-core form, else 0
  int spread_pmax = 1;  // largest stencil width P of the list
  Segs seg{};
  // per-system vectors (pointer tables) and leading dimension of the basis
  const double **V, **bx, **by, **t1, **b, **x2, **r, **irr, **ird;
  size_t *ld;
  double *ones, *zeros, *mones;
  char *dev = nullptr;
  size_t cap = 0;
  int signature = -1;
};

}  // namespace

struct BatchEngine {
  std::vector<fbim_ctx *> sys;
  hipStream_t stream = nullptr;
  bool mixed = false;
  bool basis32 = false;  // GMRES basis columns stored as FP32 (mixed engines, FBIM_FLAG_BASIS32)
  bool conv = false;  // fused transform kernels for every system (else rocFFT plans per class)
  uint32_t flags = 0;
  std::vector<SizeClass> classes;
  std::vector<int> cls_of, slot_of;
  rocfft_execution_info einfo = nullptr;
  void *work = nullptr;
  size_t work_bytes = 0;
  static constexpr int kSubSlots = 8;
  Tables full, sub[kSubSlots];  // the full list and recent sub-lists (filled in turn)
  int sub_next = 0;
  double *d_sc = nullptr;  // per-system scalars: [a | h | h2 | nrm | flag | c] blocks
  size_t sc_cap = 0;
  int hs = 0;
  double *d_partial = nullptr;
  size_t partial_cap = 0;
  // lagged reorthogonalisation: the previous lagged-pass outputs of the systems of
  // the next pass, uploaded in table order (pinned staging, kLagSlot per system)
  double *d_lagin = nullptr, *h_lagin = nullptr;
  size_t lag_cap = 0;
  HostPub pub;  // per-system orthogonalisation results and norms read by the host
  // graphs of the precond + operator launch set per table slot (full, then
  // sub[]) and precision, with the launch arguments they were captured with
  hipGraphExec_t gexec[1 + kSubSlots][2] = {};
  std::vector<uint64_t> gsig[1 + kSubSlots][2];
  hipStream_t cap_stream = nullptr;  // private stream for graph capture (the null stream cannot capture)
  std::string err;
};

namespace {

fbim_status efail(BatchEngine *E, fbim_status s, const std::string &m) {
  E->err = m;
  return s;
}

#define EHIP(E, expr)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return efail(E, FBIM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define EFFT(E, expr)                                                                             \
  do {                                                                                            \
    rocfft_status e_ = (expr);                                                                    \
    if (e_ != rocfft_status_success)                                                              \
      return efail(E, FBIM_EDEVICE, std::string(#expr) + ": rocfft status " + std::to_string((int)e_)); \
  } while (0)

#define EST(expr)                 \
  do {                            \
    fbim_status s_ = (expr);      \
    if (s_ != FBIM_OK) return s_; \
  } while (0)

WaveArgs wave_args(const fbim_ctx *c) { return c->wave(); }

void destroy_classes(BatchEngine *E) {
  for (auto &k : E->classes) {
    if (k.fwd) rocfft_plan_destroy(k.fwd);
    if (k.inv) rocfft_plan_destroy(k.inv);
    if (k.fwd32) rocfft_plan_destroy(k.fwd32);
    if (k.inv32) rocfft_plan_destroy(k.inv32);
    dfree(k.grid);
    dfree(k.spec);
    dfree(k.grid32);
    dfree(k.spec32);
  }
  E->classes.clear();
}

void destroy_graphs(BatchEngine *E) {
  for (int i = 0; i <= BatchEngine::kSubSlots; ++i)
    for (int j = 0; j < 2; ++j) {
      if (E->gexec[i][j]) hipGraphExecDestroy(E->gexec[i][j]);
      E->gexec[i][j] = nullptr;
      E->gsig[i][j].clear();
    }
}

// FFT size classes and their plans (rebuilt only when the grouping changes)
fbim_status setup_classes(BatchEngine *E) {
  std::vector<int> Ms;
  for (auto *c : E->sys) Ms.push_back(c->d.M);
  std::vector<SizeClass> want;
  std::vector<int> cls(E->sys.size()), slot(E->sys.size());
  for (size_t i = 0; i < E->sys.size(); ++i) {
    int k = -1;
    for (size_t j = 0; j < want.size(); ++j)
      if (want[j].M == Ms[i]) k = (int)j;
    if (k < 0) {
      want.push_back(SizeClass{});
      want.back().M = Ms[i];
      k = (int)want.size() - 1;
    }
    cls[i] = k;
    slot[i] = (int)want[k].sys.size();
    want[k].sys.push_back((int)i);
  }
  // the fused transform kernels serve the batch when they serve every system
  bool conv = true;
  for (auto *c : E->sys) conv = conv && c->conv;
  bool same = want.size() == E->classes.size() && conv == E->conv;
  for (size_t j = 0; same && j < want.size(); ++j)
    same = want[j].M == E->classes[j].M && want[j].sys == E->classes[j].sys;
  E->cls_of = cls;
  E->slot_of = slot;
  if (same) return FBIM_OK;
  destroy_graphs(E);
  destroy_classes(E);
  E->conv = conv;
  if (conv) {
    for (auto &k : want) {
      const size_t M = k.M, cnt = k.sys.size();
      EHIP(E, dalloc(k.grid, 2 * M * M * cnt));
      EHIP(E, dalloc(k.spec, 4 * M * (M / 2 + 1) * cnt));
      if (E->mixed) {
        EHIP(E, dalloc(k.grid32, 2 * M * M * cnt));
        EHIP(E, dalloc(k.spec32, 4 * M * (M / 2 + 1) * cnt));
      }
    }
    E->classes = want;
    return FBIM_OK;
  }
  if (!g_rocfft_ready) {
    EFFT(E, rocfft_setup());
    g_rocfft_ready = true;
  }
  size_t wmax = 0;
  for (auto &k : want) {
    const size_t M = k.M, cnt = k.sys.size();
    const size_t len[2] = {M, M};
    auto plan = [&](rocfft_plan *p, rocfft_transform_type t, rocfft_precision pr) -> fbim_status {
      EFFT(E, rocfft_plan_create(p, rocfft_placement_notinplace, t, pr, 2, len, 2 * cnt, nullptr));
      size_t w = 0;
      EFFT(E, rocfft_plan_get_work_buffer_size(*p, &w));
      wmax = std::max(wmax, w);
      return FBIM_OK;
    };
    EST(plan(&k.fwd, rocfft_transform_type_real_forward, rocfft_precision_double));
    EST(plan(&k.inv, rocfft_transform_type_real_inverse, rocfft_precision_double));
    EHIP(E, dalloc(k.grid, 2 * M * M * cnt));
    EHIP(E, dalloc(k.spec, 4 * M * (M / 2 + 1) * cnt));
    if (E->mixed) {
      EST(plan(&k.fwd32, rocfft_transform_type_real_forward, rocfft_precision_single));
      EST(plan(&k.inv32, rocfft_transform_type_real_inverse, rocfft_precision_single));
      EHIP(E, dalloc(k.grid32, 2 * M * M * cnt));
      EHIP(E, dalloc(k.spec32, 4 * M * (M / 2 + 1) * cnt));
    }
  }
  E->classes = want;
  if (!E->einfo) EFFT(E, rocfft_execution_info_create(&E->einfo));
  if (wmax > E->work_bytes) {
    if (E->work) hipFree(E->work);
    E->work = nullptr;
    EHIP(E, hipMalloc(&E->work, wmax));
    E->work_bytes = wmax;
  }
  if (E->work_bytes) EFFT(E, rocfft_execution_info_set_work_buffer(E->einfo, E->work, E->work_bytes));
  EFFT(E, rocfft_execution_info_set_stream(E->einfo, E->stream));
  return FBIM_OK;
}

// build (and upload) the job tables of the systems `list` (engine indices)
fbim_status build_tables(BatchEngine *E, const std::vector<int> &list, Tables &T) {
  const int S = (int)list.size();
  // host images
  std::vector<GatherJob> gc[2], gt[2];
  std::vector<PairJob> pj[2];
  std::vector<AlpertJob> aj;
  std::vector<SpreadJob> sj[2];
  std::vector<MultJob> mj[2];
  std::vector<InterpJob> ij[2];
  std::vector<RigidJob> rj;
  std::vector<PrecondJob> pr;
  std::vector<int> b_nodes{0}, b_pair{0}, b_tiles{0}, b_spec{0}, b_bod{0}, b_prec{0};
  std::vector<int2> chunks;
  std::vector<int> chunk_sys, sys_chunk{0};
  std::vector<const double *> V, bx, by, t1, bb, x2, r, irr, ird;
  std::vector<size_t> ld;
  size_t lds = 0;
  for (int q = 0; q < S; ++q) {
    fbim_ctx *c = E->sys[list[q]];
    const SizeClass &k = E->classes[E->cls_of[list[q]]];
    const int slot = E->slot_of[list[q]];
    const size_t M = c->d.M, gsz = 2 * M * M, ssz = 4 * M * (M / 2 + 1);
    for (int p = 0; p < 2; ++p) {
      const bool f = p == 1;
      gc[p].push_back(GatherJob{c->N, c->d_cperm, c->d_t1, f ? (void *)c->d_src32 : (void *)c->d_src64, 1});
      gt[p].push_back(GatherJob{c->N, c->d_tperm, c->d_t1, f ? (void *)c->d_mut32 : (void *)c->d_mut, 0});
      PairJob j;
      j.N = c->N;
      j.ngroups = c->ngroups;
      j.perm = c->d_cperm;
      j.goff = c->d_goff;
      j.gnn = c->d_gnn;
      j.gnf = c->d_gnf;
      j.ell = c->d_ell;
      j.tcell = c->d_tcell;
      j.cell_start = c->d_cstart;
      j.nb = c->d.n_box;
      j.cell = c->d.L / c->d.n_box;
      j.xi2 = c->d.xi * c->d.xi;
      j.cG = 1.0 / (4.0 * kPi * c->p.eta);
      j.src = f ? (const void *)c->d_src32 : (const void *)c->d_src64;
      j.out = c->d_by;
      pj[p].push_back(j);
      const WaveArgs w = wave_args(c);
      void *grid = f ? (void *)(k.grid32 + slot * gsz) : (void *)(k.grid + slot * gsz);
      void *spec = f ? (void *)(k.spec32 + slot * ssz) : (void *)(k.spec + slot * ssz);
      sj[p].push_back(SpreadJob{w, f ? (const void *)c->d_xt32 : (const void *)c->d_xt,
                                f ? (const void *)c->d_mut32 : (const void *)c->d_mut, grid});
      mj[p].push_back(MultJob{(int)M, c->d.L, c->d.xi, c->d.eta_s, c->d.h * c->d.h / (c->p.eta * c->d.L * c->d.L),
                              spec});
      ij[p].push_back(InterpJob{w, f ? (const void *)c->d_xt32 : (const void *)c->d_xt, c->d_tperm, grid, c->d_by});
    }
    aj.push_back(AlpertJob{c->geom(), c->d_band_arr, c->d_band, c->d_t1, c->d_by});
    rj.push_back(RigidJob{c->geom(), c->d_t1, c->d_by});
    pr.push_back(PrecondJob{c->geom(), c->mats(), c->bt, c->mlp_on ? c->d_dN : nullptr, c->d_bx, c->d_t1});
    b_nodes.push_back(b_nodes.back() + (c->N + 255) / 256);
    b_pair.push_back(b_pair.back() + c->ngroups);  // one work group per group of 64 targets
    b_tiles.push_back(b_tiles.back() + c->nts * c->nts);
    b_spec.push_back(b_spec.back() + (int)((M * (M / 2 + 1) + 255) / 256));
    b_bod.push_back(b_bod.back() + (c->n + 3) / 4);
    b_prec.push_back(b_prec.back() + c->bt.ntile);
    lds = std::max(lds, c->bt.lds_bytes);
    for (size_t x = 0; x < c->ntot; x += kChunk) {
      chunks.push_back(make_int2((int)x, (int)std::min(c->ntot, x + kChunk)));
      chunk_sys.push_back(q);
    }
    sys_chunk.push_back((int)chunks.size());
    V.push_back(c->d_V);
    bx.push_back(c->d_bx);
    by.push_back(c->d_by);
    t1.push_back(c->d_t1);
    bb.push_back(c->d_b);
    x2.push_back(c->d_x2);
    r.push_back(c->d_r);
    irr.push_back(c->d_irr);
    ird.push_back(c->d_ird);
    ld.push_back(c->ntot);
  }
  // pack: sizes first
  size_t off = 0;
  char *null = nullptr;
  auto plan_layout = [&](char *base) {
    off = 0;
    for (int p = 0; p < 2; ++p) {
      T.gcell[p] = carve<GatherJob>(base, off, S);
      T.gtile[p] = carve<GatherJob>(base, off, S);
      T.pair[p] = carve<PairJob>(base, off, S);
      T.spr[p] = carve<SpreadJob>(base, off, S);
      T.mul[p] = carve<MultJob>(base, off, S);
      T.itp[p] = carve<InterpJob>(base, off, S);
    }
    T.alp = carve<AlpertJob>(base, off, S);
    T.rig = carve<RigidJob>(base, off, S);
    T.pre = carve<PrecondJob>(base, off, S);
    T.bg_nodes.begin = carve<int>(base, off, S + 1);
    T.bg_pair.begin = carve<int>(base, off, S + 1);
    T.bg_tiles.begin = carve<int>(base, off, S + 1);
    T.bg_spec.begin = carve<int>(base, off, S + 1);
    T.bg_bodies4.begin = carve<int>(base, off, S + 1);
    T.bg_prec.begin = carve<int>(base, off, S + 1);
    T.seg.chunk = carve<int2>(base, off, chunks.size());
    T.seg.chunk_sys = carve<int>(base, off, chunks.size());
    T.seg.sys_chunk = carve<int>(base, off, S + 1);
    T.V = carve<const double *>(base, off, S);
    T.bx = carve<const double *>(base, off, S);
    T.by = carve<const double *>(base, off, S);
    T.t1 = carve<const double *>(base, off, S);
    T.b = carve<const double *>(base, off, S);
    T.x2 = carve<const double *>(base, off, S);
    T.r = carve<const double *>(base, off, S);
    T.irr = carve<const double *>(base, off, S);
    T.ird = carve<const double *>(base, off, S);
    T.ld = carve<size_t>(base, off, S);
    T.ones = carve<double>(base, off, S);
    T.zeros = carve<double>(base, off, S);
    T.mones = carve<double>(base, off, S);
  };
  plan_layout(null);
  const size_t bytes = off + 256;
  if (bytes > T.cap) {
    if (T.dev) hipFree(T.dev);
    T.dev = nullptr;
    EHIP(E, hipMalloc((void **)&T.dev, bytes));
    T.cap = bytes;
  }
  std::vector<char> host(bytes, 0);
  plan_layout(host.data());
  auto put = [&](const void *dst_in_host, const void *src, size_t n) {
    std::memcpy(const_cast<void *>(dst_in_host), src, n);
  };
  for (int p = 0; p < 2; ++p) {
    put(T.gcell[p], gc[p].data(), S * sizeof(GatherJob));
    put(T.gtile[p], gt[p].data(), S * sizeof(GatherJob));
    put(T.pair[p], pj[p].data(), S * sizeof(PairJob));
    put(T.spr[p], sj[p].data(), S * sizeof(SpreadJob));
    put(T.mul[p], mj[p].data(), S * sizeof(MultJob));
    put(T.itp[p], ij[p].data(), S * sizeof(InterpJob));
  }
  put(T.alp, aj.data(), S * sizeof(AlpertJob));
  put(T.rig, rj.data(), S * sizeof(RigidJob));
  put(T.pre, pr.data(), S * sizeof(PrecondJob));
  put(T.bg_nodes.begin, b_nodes.data(), (S + 1) * sizeof(int));
  put(T.bg_pair.begin, b_pair.data(), (S + 1) * sizeof(int));
  put(T.bg_tiles.begin, b_tiles.data(), (S + 1) * sizeof(int));
  put(T.bg_spec.begin, b_spec.data(), (S + 1) * sizeof(int));
  put(T.bg_bodies4.begin, b_bod.data(), (S + 1) * sizeof(int));
  put(T.bg_prec.begin, b_prec.data(), (S + 1) * sizeof(int));
  put(T.seg.chunk, chunks.data(), chunks.size() * sizeof(int2));
  put(T.seg.chunk_sys, chunk_sys.data(), chunks.size() * sizeof(int));
  put(T.seg.sys_chunk, sys_chunk.data(), (S + 1) * sizeof(int));
  put(T.V, V.data(), S * sizeof(double *));
  put(T.bx, bx.data(), S * sizeof(double *));
  put(T.by, by.data(), S * sizeof(double *));
  put(T.t1, t1.data(), S * sizeof(double *));
  put(T.b, bb.data(), S * sizeof(double *));
  put(T.x2, x2.data(), S * sizeof(double *));
  put(T.r, r.data(), S * sizeof(double *));
  put(T.irr, irr.data(), S * sizeof(double *));
  put(T.ird, ird.data(), S * sizeof(double *));
  put(T.ld, ld.data(), S * sizeof(size_t));
  std::vector<double> ones(S, 1.0), zeros(S, 0.0), mones(S, -1.0);
  put(T.ones, ones.data(), S * sizeof(double));
  put(T.zeros, zeros.data(), S * sizeof(double));
  put(T.mones, mones.data(), S * sizeof(double));
  EHIP(E, hipMemcpyAsync(T.dev, host.data(), bytes, hipMemcpyHostToDevice, E->stream));
  EHIP(E, hipStreamSynchronize(E->stream));  // the host image is released on return
  // rebase the layout onto the device allocation
  plan_layout(T.dev);
  T.S = S;
  T.list = list;
  T.bg_nodes.S = T.bg_pair.S = T.bg_tiles.S = T.bg_spec.S = T.bg_bodies4.S = T.bg_prec.S = S;
  T.bg_nodes.nblocks = b_nodes.back();
  T.bg_pair.nblocks = b_pair.back();
  T.bg_tiles.nblocks = b_tiles.back();
  T.bg_spec.nblocks = b_spec.back();
  T.bg_bodies4.nblocks = b_bod.back();
  T.bg_prec.nblocks = b_prec.back();
  T.prec_lds = lds;
  // the largest row-block count of the list, 0 if a system lacks the matrix-core form
  T.prec_mfma = 0;
  bool all_mfma = true;
  for (int i : list) {
    all_mfma = all_mfma && E->sys[i]->bt.mfma > 0;
    T.prec_mfma = std::max(T.prec_mfma, E->sys[i]->bt.mfma);
  }
  if (!all_mfma) T.prec_mfma = 0;
  T.spread_pmax = 1;
  for (int i : list) T.spread_pmax = std::max(T.spread_pmax, E->sys[i]->d.P);
  T.seg.nchunk = (int)chunks.size();
  T.seg.S = S;
  return FBIM_OK;
}

fbim_status ensure_batch_buffers(BatchEngine *E, fbim_ctx *c) {
  if (!c->have_bodies) return efail(E, FBIM_EINVAL, "a batch system has no bodies");
  if (c->mixed != E->mixed) return efail(E, FBIM_EINVAL, "batch systems must share the precision");
  if (c->cap_bxy != c->ntot) {
    EHIP(E, dalloc(c->d_bx, c->ntot));
    EHIP(E, dalloc(c->d_by, c->ntot));
    c->cap_bxy = c->ntot;
  }
  return FBIM_OK;
}

// (re)build everything for the engine's current system list
fbim_status engine_prepare(BatchEngine *E) {
  if (E->sys.empty()) return efail(E, FBIM_EINVAL, "empty batch");
  E->mixed = E->sys[0]->mixed;
  E->basis32 = E->mixed;
  for (auto *c : E->sys) E->basis32 = E->basis32 && (c->p.flags & FBIM_FLAG_BASIS32);
  for (auto *c : E->sys) {
    c->stream = E->stream;
    if (c->einfo) rocfft_execution_info_set_stream(c->einfo, E->stream);
    EST(ensure_batch_buffers(E, c));
  }
  EST(setup_classes(E));
  std::vector<int> all(E->sys.size());
  for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
  const void *old = E->full.dev;
  const int oldS = E->full.S;
  const int oldb[3] = {E->full.bg_pair.nblocks, E->full.bg_tiles.nblocks, E->full.bg_prec.nblocks};
  EST(build_tables(E, all, E->full));
  // sub-lists are rebuilt in the order of first use, so a launch sequence that
  // repeats lands on the same slots (and graphs) again
  for (auto &t : E->sub) t.list.clear();
  E->sub_next = 0;
  // per-system scalar blocks (sized for the full list) and reduction partials
  E->hs = 0;
  for (auto *c : E->sys) E->hs = std::max(E->hs, (int)c->capV + 2);
  const size_t need = E->sys.size() * (3 * (size_t)E->hs + 8);
  if (need > E->sc_cap) {
    EHIP(E, dalloc(E->d_sc, need));
    E->sc_cap = need;
  }
  EHIP(E, pub_alloc(E->pub, E->sys.size() * std::max((size_t)E->hs + 1, (size_t)2 * kLagSlot)));
  if (E->sys.size() * (size_t)kLagSlot > E->lag_cap) {
    if (E->h_lagin) hipHostFree(E->h_lagin);
    E->h_lagin = nullptr;
    E->lag_cap = 0;
    EHIP(E, dalloc(E->d_lagin, E->sys.size() * (size_t)kLagSlot));
    EHIP(E, hipHostMalloc((void **)&E->h_lagin, E->sys.size() * kLagSlot * sizeof(double), hipHostMallocDefault));
    E->lag_cap = E->sys.size() * (size_t)kLagSlot;
  }
  const size_t pneed = (size_t)std::max(E->full.seg.nchunk, 1) * (E->hs + 1);
  if (pneed > E->partial_cap) {
    EHIP(E, dalloc(E->d_partial, pneed));
    E->partial_cap = pneed;
  }
  const bool same = old == E->full.dev && oldS == E->full.S && oldb[0] == E->full.bg_pair.nblocks &&
                    oldb[1] == E->full.bg_tiles.nblocks && oldb[2] == E->full.bg_prec.nblocks;
  if (!same) destroy_graphs(E);
  return FBIM_OK;
}

Tables &tables_for(BatchEngine *E, const std::vector<int> &list, fbim_status &st) {
  st = FBIM_OK;
  if (list == E->full.list) return E->full;
  for (auto &t : E->sub)
    if (list == t.list) return t;
  Tables &t = E->sub[E->sub_next];
  E->sub_next = (E->sub_next + 1) % BatchEngine::kSubSlots;
  st = build_tables(E, list, t);
  return t;
}

// ---------------------------------------------------------------- batched operators
// y = P^-1 bx for every system of T (into t1)
fbim_status run_precond(BatchEngine *E, Tables &T) {
  Timer t(E->sys[0], "precond");
  EHIP(E, launch_precond_batch(T.pre, T.bg_prec, T.prec_lds, T.prec_mfma, E->stream));
  return FBIM_OK;
}

// by = M t1 (and the rigid-body rows of the saddle operator when saddle != 0)
fbim_status run_operator(BatchEngine *E, Tables &T, bool f32, bool saddle) {
  hipStream_t s = E->stream;
  fbim_ctx *tc = E->sys[0];
  const int p = f32 ? 1 : 0;
  // the input in cell order (pair kernel) and in tile order (spreading), one launch
  EHIP(E, launch_gather2x2_batch(T.gcell[p], T.gtile[p], T.bg_nodes, p, s));
  {
    Timer t(tc, f32 ? "pair32" : "pair");
    EHIP(E, launch_pair_batch(T.pair[p], T.bg_pair, p, tc->d_e1tab, tc->d_e1tab32, s));
  }
  {
    Timer t(tc, "alpert");
    EHIP(E, launch_alpert_batch(T.alp, T.bg_nodes, s));
  }
  {
    Timer t(tc, f32 ? "spread32" : "spread");
    EHIP(E, launch_spread_batch(T.spr[p], T.bg_tiles, p, T.spread_pmax, s));
  }
  if (E->conv) {
    // fused transform kernels, per listed system on its slot of the class buffers
    Timer t(tc, f32 ? "fft32" : "fft");
    for (int q = 0; q < T.S; ++q) {
      fbim_ctx *c = E->sys[T.list[q]];
      const SizeClass &k = E->classes[E->cls_of[T.list[q]]];
      const size_t M = c->d.M, slot = E->slot_of[T.list[q]], gsz = 2 * M * M, ssz = 4 * M * (M / 2 + 1);
      const WaveConvArgs a{c->d.M, 0, c->d.L, c->d.xi, c->d.eta_s, c->d.h * c->d.h / (c->p.eta * c->d.L * c->d.L)};
      if (f32)
        EHIP(E, launch_wave_conv_f32(a, k.grid32 + slot * gsz, k.spec32 + slot * ssz, c->d_tw32, c->d_ey32, s));
      else
        EHIP(E, launch_wave_conv_f64(a, k.grid + slot * gsz, k.spec + slot * ssz, c->d_tw, c->d_ey, s));
    }
  } else {
    {
      Timer t(tc, f32 ? "fft32" : "fft");
      for (auto &k : E->classes) {
        void *in[1] = {f32 ? (void *)k.grid32 : (void *)k.grid}, *o[1] = {f32 ? (void *)k.spec32 : (void *)k.spec};
        EFFT(E, rocfft_execute(f32 ? k.fwd32 : k.fwd, in, o, E->einfo));
      }
    }
    {
      Timer t(tc, f32 ? "multiplier32" : "multiplier");
      EHIP(E, launch_multiplier_batch(T.mul[p], T.bg_spec, p, 0, s));
    }
    Timer t(tc, f32 ? "fft32" : "fft");
    for (auto &k : E->classes) {
      void *in[1] = {f32 ? (void *)k.spec32 : (void *)k.spec}, *o[1] = {f32 ? (void *)k.grid32 : (void *)k.grid};
      EFFT(E, rocfft_execute(f32 ? k.inv32 : k.inv, in, o, E->einfo));
    }
  }
  {
    Timer t(tc, f32 ? "interp32" : "interp");
    EHIP(E, launch_interp_batch(T.itp[p], T.bg_tiles, p, T.spread_pmax, s));
  }
  if (saddle) EHIP(E, launch_rigid_batch(T.rig, T.bg_nodes, T.bg_bodies4, s));
  return FBIM_OK;
}

// Everything the precond + operator launches of T take by value: a graph
// captured with one signature replays correctly while the signature holds (the
// tables themselves are read from device memory at replay).
std::vector<uint64_t> launch_signature(const BatchEngine *E, const Tables &T) {
  std::vector<uint64_t> v;
  auto P = [&](const void *p) { v.push_back((uint64_t)(uintptr_t)p); };
  auto D = [&](double x) {
    uint64_t u;
    std::memcpy(&u, &x, sizeof u);
    v.push_back(u);
  };
  v.push_back((uint64_t)T.S);
  for (int i : T.list) v.push_back((uint64_t)i);
  P(T.dev);
  for (int p = 0; p < 2; ++p) {
    P(T.gcell[p]);
    P(T.gtile[p]);
    P(T.pair[p]);
    P(T.spr[p]);
    P(T.mul[p]);
    P(T.itp[p]);
  }
  P(T.alp);
  P(T.rig);
  P(T.pre);
  for (const BatchGrid *g : {&T.bg_nodes, &T.bg_pair, &T.bg_tiles, &T.bg_spec, &T.bg_bodies4, &T.bg_prec}) {
    P(g->begin);
    v.push_back(((uint64_t)(uint32_t)g->S << 32) | (uint32_t)g->nblocks);
  }
  v.push_back(T.prec_lds);
  v.push_back((uint64_t)T.prec_mfma);
  v.push_back((uint64_t)T.spread_pmax);
  P(E->sys[0]->d_e1tab);
  P(E->sys[0]->d_e1tab32);
  P(E->work);
  P(E->einfo);
  v.push_back(E->conv ? 1 : 0);
  for (const SizeClass &k : E->classes) {
    P(k.grid);
    P(k.spec);
    P(k.grid32);
    P(k.spec32);
    P(k.fwd);
    P(k.inv);
    P(k.fwd32);
    P(k.inv32);
  }
  for (int i : T.list) {
    const fbim_ctx *c = E->sys[i];
    v.push_back(((uint64_t)(uint32_t)E->cls_of[i] << 32) | (uint32_t)E->slot_of[i]);
    P(c->d_tw);
    P(c->d_ey);
    P(c->d_tw32);
    P(c->d_ey32);
    v.push_back((uint64_t)c->d.M);
    for (double x : {c->d.L, c->d.xi, c->d.eta_s, c->d.h, c->p.eta}) D(x);
  }
  return v;
}

// t1 = P^-1 bx, by = A t1 for every system of T; replayed from a HIP graph
// (one per table slot and precision) when enabled and graph_ok
fbim_status run_precond_saddle(BatchEngine *E, Tables &T, bool f32, bool graph_ok = true) {
  const bool graph = graph_ok && (E->flags & FBIM_BATCH_GRAPH) && !E->sys[0]->timing;
  if (!graph) {
    EST(run_precond(E, T));
    return run_operator(E, T, f32, true);
  }
  const int ti = &T == &E->full ? 0 : 1 + (int)(&T - E->sub);
  const int gi = f32 ? 1 : 0;
  hipGraphExec_t &ge = E->gexec[ti][gi];
  std::vector<uint64_t> sig = launch_signature(E, T);
  if (ge && sig != E->gsig[ti][gi]) {
    hipGraphExecDestroy(ge);
    ge = nullptr;
  }
  if (!ge) {
    if (!E->cap_stream) EHIP(E, hipStreamCreateWithFlags(&E->cap_stream, hipStreamNonBlocking));
    // capture on the private stream (nothing runs during capture), then launch on ours
    EHIP(E, hipStreamSynchronize(E->stream));
    hipStream_t user = E->stream;
    E->stream = E->cap_stream;
    if (E->einfo) rocfft_execution_info_set_stream(E->einfo, E->stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal);
    fbim_status st = e == hipSuccess ? run_precond(E, T) : FBIM_EDEVICE;
    if (st == FBIM_OK) st = run_operator(E, T, f32, true);
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(E->stream, &g) : e;
    E->stream = user;
    if (E->einfo) rocfft_execution_info_set_stream(E->einfo, E->stream);
    if (st != FBIM_OK) {
      if (g) hipGraphDestroy(g);
      return st == FBIM_EDEVICE && e != hipSuccess ? efail(E, st, "hipStreamBeginCapture failed") : st;
    }
    EHIP(E, e2);
    // memset nodes replay unreliably here: keep such a graph out and run eagerly
    size_t nn = 0;
    EHIP(E, hipGraphGetNodes(g, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    if (nn) EHIP(E, hipGraphGetNodes(g, nodes.data(), &nn));
    bool memset_node = false;
    for (auto nd : nodes) {
      hipGraphNodeType ty;
      if (hipGraphNodeGetType(nd, &ty) == hipSuccess && ty == hipGraphNodeTypeMemset) memset_node = true;
    }
    if (memset_node) {
      hipGraphDestroy(g);
      E->flags &= ~FBIM_BATCH_GRAPH;
      EST(run_precond(E, T));
      return run_operator(E, T, f32, true);
    }
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    EHIP(E, e);
    E->gsig[ti][gi] = std::move(sig);
  }
  EHIP(E, hipGraphLaunch(ge, E->stream));
  return FBIM_OK;
}

// ---------------------------------------------------------------- Krylov helpers
VecRef vref(const double **base, int col = 0, const size_t *ld = nullptr) {
  VecRef v;
  v.base = base;
  v.ld = ld;
  v.col = col;
  return v;
}

// column `col` of every system's GMRES basis (FP32 columns on FP32-basis engines;
// the leading dimension then counts floats, so the columns fill half the storage)
VecRef vbasis(const BatchEngine *E, const Tables &T, int col) {
  VecRef v = vref(T.V, col, T.ld);
  v.f32 = E->basis32 ? 1 : 0;
  return v;
}

fbim_status seg_axpby(BatchEngine *E, Tables &T, VecRef x, VecRef y, const double *a, const double *b) {
  Timer t(E->sys[0], "blas");
  EHIP(E, launch_seg_axpby(T.seg, x, y, a, b, E->stream));
  return FBIM_OK;
}

struct Scal {
  double *a, *h, *h2, *nrm, *flag, *c;
};
// per-system scalar blocks for a table of S systems (table order)
Scal scalars(BatchEngine *E, int S) {
  Scal q;
  double *p = E->d_sc;
  q.a = p;
  p += S;
  q.h = p;
  p += (size_t)S * E->hs;
  q.h2 = p;
  p += (size_t)S * E->hs;
  q.nrm = p;
  p += (size_t)S * 4;
  q.flag = p;
  p += S;
  q.c = p;
  return q;
}

fbim_status orth_pass_b(BatchEngine *E, Tables &T, int mode, int k, const double **w, const double *h,
                        const double *cond, double *out, int ostride) {
  Timer t(E->sys[0], "blas");
  OrthArgs a;
  a.seg = T.seg;
  a.V = nullptr;
  a.ld = 0;
  a.k = k;
  a.w = nullptr;
  a.Vs = T.V;
  a.v32 = E->basis32 ? 1 : 0;
  a.ws = const_cast<double *const *>(w);
  a.lds = T.ld;
  a.h = h;
  a.hstride = E->hs;
  a.cond = cond;
  a.partial = E->d_partial;
  a.out = out;
  a.ostride = ostride;
  EHIP(E, launch_orth(mode, a, E->stream));
  return FBIM_OK;
}

// squared norms of w_s, host, table order
fbim_status norms_b(BatchEngine *E, Tables &T, const double **w, std::vector<double> &nrm2) {
  Scal q = scalars(E, T.S);
  EST(orth_pass_b(E, T, 0, 0, w, nullptr, nullptr, q.nrm, 4));
  const unsigned long long tag = ++E->pub.seq;
  EHIP(E, launch_publish(T.S, q.nrm, 4, E->pub, tag, E->stream));
  EHIP(E, pub_wait(E->pub, tag, E->stream));
  nrm2.assign(E->pub.v, E->pub.v + T.S);
  return FBIM_OK;
}

fbim_status upload_a(BatchEngine *E, const std::vector<double> &a) {
  EHIP(E, hipMemcpyAsync(E->d_sc, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice, E->stream));
  EHIP(E, hipStreamSynchronize(E->stream));  // the host vector may be released on return
  return FBIM_OK;
}

// CGS2 (or DGKS-selective) orthogonalisation of by_s against V_s[:, 0..k) for
// every system of T; h[q][0..k) (host) and hn[q] = ||by_s|| afterwards.  With
// `next`, next_s = by_s / hn_s (0 where hn_s = 0) is written, and its FP64 copy
// into bx_s (the preconditioner's input of the next iteration), before the host
// waits: the device finds the scales itself.
fbim_status orthogonalise_b(BatchEngine *E, Tables &T, int k, std::vector<std::vector<double>> &h,
                            std::vector<double> &hn, const VecRef *next = nullptr) {
  const int S = T.S, hs = E->hs;
  Scal q = scalars(E, S);
  const bool selective = (E->sys[0]->p.flags & FBIM_FLAG_SELECTIVE_REORTH) != 0;
  const bool fused = k <= kOrthFused;
  EST(orth_pass_b(E, T, 0, k, T.by, nullptr, nullptr, q.h, hs));
  if (fused) {
    EST(orth_pass_b(E, T, 1, k, T.by, q.h, nullptr, q.h2, hs));
    if (selective) EHIP(E, launch_need_second_pass(S, q.h2 + k, hs, q.h + k, hs, q.flag, E->stream));
    EST(orth_pass_b(E, T, 2, k, T.by, q.h2, selective ? q.flag : nullptr, q.nrm + 2, 4));
  } else {
    EST(orth_pass_b(E, T, 2, k, T.by, q.h, nullptr, q.nrm, 4));
    if (selective) EHIP(E, launch_need_second_pass(S, q.nrm, 4, q.h + k, hs, q.flag, E->stream));
    EST(orth_pass_b(E, T, 0, k, T.by, nullptr, selective ? q.flag : nullptr, q.h2, hs));
    EST(orth_pass_b(E, T, 2, k, T.by, q.h2, selective ? q.flag : nullptr, q.nrm + 2, 4));
  }
  OrthPublish o;
  o.S = S;
  o.k = k;
  o.hs = hs;
  o.ns = 4;
  o.fs = 1;
  o.as = 1;
  o.fused = fused;
  o.selective = selective;
  o.h = q.h;
  o.h2 = q.h2;
  o.nrm_a = q.nrm;
  o.nrm_b = q.nrm + 2;
  o.flag = q.flag;
  o.a = q.a;
  const unsigned long long tag = ++E->pub.seq;
  EHIP(E, launch_orth_publish(o, E->pub, tag, E->stream));
  if (next) {
    Timer t(E->sys[0], "blas");
    EHIP(E, launch_seg_scale2(T.seg, vref(T.by), *next, vref(T.bx), q.a, E->stream));
  }
  EHIP(E, pub_wait(E->pub, tag, E->stream));
  const double *v = E->pub.v;
  h.assign(S, std::vector<double>(k));
  hn.assign(S, 0.0);
  for (int i = 0; i < S; ++i) {
    std::memcpy(h[i].data(), v + (size_t)i * (k + 1), k * sizeof(double));
    hn[i] = v[(size_t)i * (k + 1) + k];
  }
  return FBIM_OK;
}

// One lockstep Arnoldi step with delayed reorthogonalisation (FBIM_FLAG_LAGGED_REORTH)
// for the systems of T: the dot-product pass and the lagged pass run over basis slots
// 0..j and w = by; the lagged pass finalises slot j and writes the new vector w',
// unnormalised, to slot j + 1 and its FP64 copy to bx (the next operator input).  The
// lagged pass reads each system's previous lagged-pass output (j + 1 values)
// where the previous step left it when it ran on the same systems in the same table
// order (`same`), else from lagprev (host, table order) through a pinned upload.
// dots[q] and outs[q] point to system q's published dot products and lagged-pass
// output (j + 2 values each) until the next publication.
fbim_status orthogonalise_lag_b(BatchEngine *E, Tables &T, int j, bool same,
                                const std::vector<const double *> &lagprev, std::vector<const double *> &dots,
                                std::vector<const double *> &outs) {
  const int S = T.S, hs = E->hs;
  Scal q = scalars(E, S);
  if (j > 0 && !same) {
    // the staging buffer's previous copy ran before the last publication the host waited for
    for (int p = 0; p < S; ++p) std::memcpy(E->h_lagin + (size_t)p * kLagSlot, lagprev[p], (j + 1) * sizeof(double));
    EHIP(E, hipMemcpyAsync(E->d_lagin, E->h_lagin, (size_t)S * kLagSlot * sizeof(double), hipMemcpyHostToDevice,
                           E->stream));
  }
  EST(orth_pass_b(E, T, 0, j + 1, T.by, nullptr, nullptr, q.h, hs));
  {
    Timer t(E->sys[0], "blas");
    OrthArgs a{};
    a.seg = T.seg;
    a.k = j;
    a.Vs = T.V;
    a.v32 = E->basis32 ? 1 : 0;
    a.ws = const_cast<double *const *>(T.by);
    a.lds = T.ld;
    a.h = q.h;
    a.hstride = hs;
    a.cond = nullptr;
    a.partial = E->d_partial;
    a.out = q.h2;
    a.ostride = hs;
    // in place: every work group reads its system's lag before the reduction launch
    // that writes this pass's output over it
    a.lag = j == 0 ? nullptr : (same ? q.h2 : E->d_lagin);
    a.lagstride = same ? hs : kLagSlot;
    a.next = 1;
    a.xs = const_cast<double *const *>(T.bx);
    EHIP(E, launch_orth_lag(a, E->stream));
  }
  const unsigned long long tag = ++E->pub.seq;
  EHIP(E, launch_publish2(S, j + 2, q.h, hs, j + 2, q.h2, hs, E->pub, tag, E->stream));
  EHIP(E, pub_wait(E->pub, tag, E->stream));
  dots.resize(S);
  outs.resize(S);
  for (int p = 0; p < S; ++p) {
    dots[p] = E->pub.v + (size_t)p * 2 * (j + 2);
    outs[p] = dots[p] + j + 2;
  }
  return FBIM_OK;
}

std::vector<int> pick(const std::vector<int> &v, const std::vector<int> &pos) {
  std::vector<int> out;
  for (int p : pos) out.push_back(v[p]);
  return out;
}

// Lockstep right-preconditioned restarted GMRES of the saddle systems `sysl`
// (engine indices): A_s x_s = rhs_s, rhs / x = (d_b, d_x2), or (d_irr, d_ird)
// when `ir`.  Every system keeps its own Krylov space, Hessenberg matrix and
// stopping test ||rhs - A x|| <= tol_s ||rhs||, and leaves the launches once
// it has converged.  Outputs per system (sysl order).
// relax > 0 (mixed engines): relaxed-matvec GMRES -- a system's iteration uses the
// FP32 operator once its residual estimate is below relax ||rhs|| (systems of both
// kinds run as two launch sets); restart residuals are FP64 (f32 is then ignored).  warm: start from the x
// given (else x = 0).
fbim_status gmres_b(BatchEngine *E, const std::vector<int> &sysl, bool ir, bool f32, const std::vector<double> &tol,
                    const std::vector<int> &maxit, std::vector<int> &iters, std::vector<double> &relres,
                    std::vector<int> &status, double relax = 0.0, bool warm = false) {
  const int S0 = (int)sysl.size();
  iters.assign(S0, 0);
  relres.assign(S0, 0.0);
  status.assign(S0, FBIM_OK);
  int m = 1 << 30;
  bool lagged = true;  // delayed reorthogonalisation when every system asks for it
  for (int i : sysl) {
    m = std::min(m, E->sys[i]->restart);
    lagged = lagged && (E->sys[i]->p.flags & FBIM_FLAG_LAGGED_REORTH);
  }
  if (lagged) m = std::min(m, kOrthFused);
  fbim_status st;
  auto rhs = [&](Tables &T) { return ir ? T.irr : T.b; };
  auto sol = [&](Tables &T) { return ir ? T.ird : T.x2; };
  Tables *T = &tables_for(E, sysl, st);
  EST(st);
  std::vector<double> nb2;
  EST(norms_b(E, *T, rhs(*T), nb2));
  std::vector<double> nb(S0);
  for (int i = 0; i < S0; ++i) {
    if (!std::isfinite(nb2[i])) return efail(E, FBIM_EINVAL, "non-finite right-hand side in a batch system");
    nb[i] = std::sqrt(std::max(nb2[i], 0.0));
  }
  if (!warm) EST(seg_axpby(E, *T, vref(sol(*T)), vref(sol(*T)), T->zeros, T->zeros));  // x = 0
  std::vector<int> running;  // positions in sysl
  for (int i = 0; i < S0; ++i)
    if (nb[i] > 0.0) running.push_back(i);
  // per-system Arnoldi state
  std::vector<std::vector<double>> H(S0), g(S0), cs(S0), sn(S0);
  // lagged: unrotated columns, lag of the newest vector, last lagged-pass output
  std::vector<std::vector<double>> Hu(S0), slag(S0), lagraw(S0);
  std::vector<double> nlag(S0, 1.0);  // norm of the newest vector as it stands in the basis
  std::vector<int> lag_act;  // the systems (positions in sysl) of the last lagged pass
  bool first = !warm;
  while (!running.empty()) {
    T = &tables_for(E, pick(sysl, running), st);
    EST(st);
    // r = rhs - A x
    EST(seg_axpby(E, *T, vref(rhs(*T)), vref(T->r), T->ones, T->zeros));
    if (!first) {
      EST(seg_axpby(E, *T, vref(sol(*T)), vref(T->t1), T->ones, T->zeros));
      EST(run_operator(E, *T, relax > 0 ? false : f32, true));
      EST(seg_axpby(E, *T, vref(T->by), vref(T->r), T->mones, T->ones));
    }
    first = false;
    std::vector<double> r2;
    EST(norms_b(E, *T, T->r, r2));
    std::vector<int> cyc;  // positions in sysl that iterate in this cycle
    std::vector<double> inv;
    for (size_t q = 0; q < running.size(); ++q) {
      const int i = running[q];
      if (!std::isfinite(r2[q])) return efail(E, FBIM_EDEVICE, "non-finite GMRES residual in a batch system");
      const double beta = std::sqrt(std::max(r2[q], 0.0));
      relres[i] = beta / nb[i];
      if (relres[i] <= tol[i]) continue;
      if (iters[i] >= maxit[i]) {
        status[i] = FBIM_ENOCONV;
        continue;
      }
      cyc.push_back(i);
      inv.push_back(1.0 / beta);
      H[i].assign((size_t)(m + 1) * m, 0.0);
      if (lagged) {
        Hu[i].assign((size_t)(m + 1) * m, 0.0);
        slag[i].clear();
        lagraw[i].clear();
        nlag[i] = 1.0;
      }
      g[i].assign(m + 1, 0.0);
      cs[i].assign(m, 0.0);
      sn[i].assign(m, 0.0);
      g[i][0] = beta;
    }
    if (cyc.empty()) break;
    T = &tables_for(E, pick(sysl, cyc), st);
    EST(st);
    EST(upload_a(E, inv));
    {  // V_0 = r / beta, and its FP64 copy into bx
      Timer t(E->sys[0], "blas");
      EHIP(E, launch_seg_scale2(T->seg, vref(T->r), vbasis(E, *T, 0), vref(T->bx), scalars(E, T->S).a, E->stream));
    }
    std::vector<int> jend(S0, 0);
    std::vector<int> act = cyc;
    for (int j = 0; j < m && !act.empty(); ++j) {
      T = &tables_for(E, pick(sysl, act), st);
      EST(st);
      // bx_s holds V_s[:, j] (written with the column)
      // relaxed: each system takes the FP32 operator once its own residual estimate
      // is below relax ||rhs|| (as it would alone); the two groups run as two launch
      // sets.  With more than two systems the groupings keep changing, so their
      // launch sets run without graphs (no capture per grouping).
      std::vector<int> p64, p32;
      if (relax > 0)
        for (int i : act) (std::fabs(g[i][j]) <= relax * nb[i] ? p32 : p64).push_back(i);
      if (relax <= 0 || p64.empty() || p32.empty()) {
        EST(run_precond_saddle(E, *T, relax > 0 ? p64.empty() : f32));
      } else {
        const bool graph_ok = act.size() <= 2;
        Tables *Tg = &tables_for(E, pick(sysl, p64), st);
        EST(st);
        EST(run_precond_saddle(E, *Tg, false, graph_ok));
        Tg = &tables_for(E, pick(sysl, p32), st);
        EST(st);
        EST(run_precond_saddle(E, *Tg, true, graph_ok));
        T = &tables_for(E, pick(sysl, act), st);
        EST(st);
      }
      std::vector<std::vector<double>> hc;
      std::vector<double> hn;
      const VecRef vnext = vbasis(E, *T, j + 1);
      if (lagged) {
        std::vector<const double *> lp(act.size()), dts, outs;
        for (size_t q = 0; q < act.size(); ++q) lp[q] = lagraw[act[q]].data();
        const bool same = j > 0 && act == lag_act;
        EST(orthogonalise_lag_b(E, *T, j, same, lp, dts, outs));  // V_j final, w' into slot j + 1 and bx
        lag_act = act;
        hc.assign(act.size(), std::vector<double>());
        hn.assign(act.size(), 0.0);
        std::vector<double> col(j + 2);
        for (size_t q = 0; q < act.size(); ++q) {
          const int i = act[q];
          if (!lagged_column(j, dts[q], outs[q], Hu[i], m, slag[i], nlag[i], col.data()))
            return efail(E, FBIM_EDEVICE, "non-finite Krylov vector in a batch system");
          for (int r = 0; r <= j + 1; ++r) Hu[i][(size_t)r * m + j] = col[r];
          lagraw[i].assign(outs[q], outs[q] + j + 2);
          hc[q].assign(col.begin(), col.begin() + j + 1);
          hn[q] = col[j + 1];
        }
      } else {
        EST(orthogonalise_b(E, *T, j + 1, hc, hn, &vnext));  // V_{j+1} = w / ||w||
      }
      std::vector<int> next;
      for (size_t q = 0; q < act.size(); ++q) {
        const int i = act[q];
        std::vector<double> col(j + 2);
        for (int r = 0; r <= j; ++r) col[r] = hc[q][r];
        col[j + 1] = hn[q];
        for (int r = 0; r < j; ++r) {  // previous rotations
          const double t1 = cs[i][r] * col[r] + sn[i][r] * col[r + 1];
          col[r + 1] = -sn[i][r] * col[r] + cs[i][r] * col[r + 1];
          col[r] = t1;
        }
        if (!std::isfinite(hn[q])) return efail(E, FBIM_EDEVICE, "non-finite Krylov vector in a batch system");
        const double den = std::hypot(col[j], col[j + 1]);
        cs[i][j] = den > 0 ? col[j] / den : 1.0;
        sn[i][j] = den > 0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        g[i][j + 1] = -sn[i][j] * g[i][j];
        g[i][j] = cs[i][j] * g[i][j];
        for (int r = 0; r <= j; ++r) H[i][(size_t)r * m + j] = col[r];
        ++iters[i];
        jend[i] = j + 1;
        const bool done = std::fabs(g[i][j + 1]) <= tol[i] * nb[i] || iters[i] >= maxit[i] || hn[q] == 0.0;
        if (!done) next.push_back(i);
      }
      act = next;
    }
    // x += P^-1 V y for the systems of this cycle
    T = &tables_for(E, pick(sysl, cyc), st);
    EST(st);
    int kmax = 0;
    for (int i : cyc) kmax = std::max(kmax, jend[i]);
    std::vector<double> c((size_t)T->S * E->hs, 0.0);
    for (size_t q = 0; q < cyc.size(); ++q) {
      const int i = cyc[q], je = jend[i];
      std::vector<double> y(je);
      for (int r = je - 1; r >= 0; --r) {
        double acc = g[i][r];
        for (int k2 = r + 1; k2 < je; ++k2) acc -= H[i][(size_t)r * m + k2] * y[k2];
        y[r] = acc / H[i][(size_t)r * m + r];
      }
      for (int r = 0; r < je; ++r) c[q * E->hs + r] = y[r];
    }
    Scal sq = scalars(E, T->S);
    EHIP(E, hipMemcpyAsync(sq.c, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, E->stream));
    {
      Timer t(E->sys[0], "blas");
      EHIP(E, launch_seg_Vc(T->seg, vbasis(E, *T, 0), kmax, sq.c, E->hs, vref(T->bx), E->stream));
    }
    EHIP(E, hipStreamSynchronize(E->stream));  // c is released on return
    EST(run_precond(E, *T));
    EST(seg_axpby(E, *T, vref(T->t1), vref(sol(*T)), T->ones, T->ones));
    running = cyc;
  }
  return FBIM_OK;
}

constexpr double kRelaxB = 1e-1;  // relaxed-matvec threshold (as for one system)

// Solve the saddle systems `sysl` with RHS d_b into d_x2.  FP64 engines: lockstep
// GMRES.  Mixed engines: relaxed-matvec lockstep GMRES, or with
// FBIM_FLAG_REFINEMENT iterative refinement as for one system -- FP64
// residuals, corrections by lockstep GMRES on the FP32 operator to 1e-3.
// warm: start from the d_x2 given (else 0).
fbim_status solve_b(BatchEngine *E, const std::vector<int> &sysl, std::vector<int> &iters, std::vector<double> &res,
                    std::vector<int> &status, bool warm = false) {
  const int S0 = (int)sysl.size();
  std::vector<double> tol(S0);
  std::vector<int> maxit(S0);
  for (int i = 0; i < S0; ++i) {
    tol[i] = E->sys[sysl[i]]->p.tol_gmres;
    maxit[i] = E->sys[sysl[i]]->gmres_max;
  }
  if (!E->mixed) return gmres_b(E, sysl, false, false, tol, maxit, iters, res, status, 0.0, warm);
  if (!(E->sys[sysl[0]]->p.flags & FBIM_FLAG_REFINEMENT))
    return gmres_b(E, sysl, false, false, tol, maxit, iters, res, status, kRelaxB, warm);
  fbim_status st;
  iters.assign(S0, 0);
  res.assign(S0, 1.0);
  status.assign(S0, FBIM_ENOCONV);
  Tables *T = &tables_for(E, sysl, st);
  EST(st);
  std::vector<double> nb2;
  EST(norms_b(E, *T, T->b, nb2));
  if (warm) {  // FP64 residual of the initial guess
    EST(seg_axpby(E, *T, vref(T->x2), vref(T->t1), T->ones, T->zeros));
    EST(run_operator(E, *T, false, true));
    EST(seg_axpby(E, *T, vref(T->b), vref(T->irr), T->ones, T->zeros));
    EST(seg_axpby(E, *T, vref(T->by), vref(T->irr), T->mones, T->ones));
  } else {
    EST(seg_axpby(E, *T, vref(T->x2), vref(T->x2), T->zeros, T->zeros));
    EST(seg_axpby(E, *T, vref(T->b), vref(T->irr), T->ones, T->zeros));
  }
  std::vector<int> running;
  for (int i = 0; i < S0; ++i) {
    if (nb2[i] > 0.0) {
      running.push_back(i);
    } else {
      res[i] = 0.0;
      status[i] = FBIM_OK;
    }
  }
  for (int outer = 0; outer < 20 && !running.empty(); ++outer) {
    std::vector<int> sl = pick(sysl, running);
    std::vector<double> itol(running.size(), 1e-3);
    std::vector<int> imax;
    for (int i : running) imax.push_back(std::max(1, maxit[i] - iters[i]));
    std::vector<int> it, ist;
    std::vector<double> ir;
    EST(gmres_b(E, sl, true, true, itol, imax, it, ir, ist));
    T = &tables_for(E, sl, st);
    EST(st);
    for (size_t q = 0; q < running.size(); ++q) iters[running[q]] += it[q];
    EST(seg_axpby(E, *T, vref(T->ird), vref(T->x2), T->ones, T->ones));
    // FP64 residual of the refined solutions
    EST(seg_axpby(E, *T, vref(T->x2), vref(T->t1), T->ones, T->zeros));
    EST(run_operator(E, *T, false, true));
    EST(seg_axpby(E, *T, vref(T->b), vref(T->irr), T->ones, T->zeros));
    EST(seg_axpby(E, *T, vref(T->by), vref(T->irr), T->mones, T->ones));
    std::vector<double> r2;
    EST(norms_b(E, *T, T->irr, r2));
    std::vector<int> next;
    for (size_t q = 0; q < running.size(); ++q) {
      const int i = running[q];
      res[i] = std::sqrt(std::max(r2[q], 0.0) / nb2[i]);
      if (res[i] <= tol[i]) {
        status[i] = FBIM_OK;
      } else if (iters[i] < maxit[i]) {
        next.push_back(i);
      }
    }
    running = next;
  }
  return FBIM_OK;
}

// b_s = -[slip_s; F_s] for one system
fbim_status rhs_one(fbim_ctx *c, const double *F, const double *slip) {
  const size_t twoN = 2 * (size_t)c->N;
  hipStream_t s = c->stream;
  if (slip)
    HIPCHK(c, launch_axpby(twoN, -1.0, slip, 0.0, c->d_b, s));
  else
    HIPCHK(c, launch_fill(twoN, 0.0, c->d_b, s));
  HIPCHK(c, launch_axpby(3 * (size_t)c->n, -1.0, F, 0.0, c->d_b + twoN, s));
  return FBIM_OK;
}

void engine_destroy(BatchEngine *E) {
  if (!E) return;
  destroy_graphs(E);
  if (E->cap_stream) hipStreamDestroy(E->cap_stream);
  destroy_classes(E);
  if (E->einfo) rocfft_execution_info_destroy(E->einfo);
  if (E->work) hipFree(E->work);
  if (E->full.dev) hipFree(E->full.dev);
  for (auto &t : E->sub)
    if (t.dev) hipFree(t.dev);
  dfree(E->d_sc);
  dfree(E->d_partial);
  dfree(E->d_lagin);
  if (E->h_lagin) hipHostFree(E->h_lagin);
  pub_free(E->pub);
  delete E;
}

fbim_status copy_out(BatchEngine *E, fbim_ctx *c, double *U) {
  EHIP(E, hipMemcpyAsync(U, c->d_x2 + 2 * (size_t)c->N, 3 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice,
                         E->stream));
  return FBIM_OK;
}

// a copy of c's shapes and parameters (for the RFD configurations)
fbim_status clone_ctx(fbim_ctx *c, fbim_ctx **out) {
  fbim_params p = c->p;
  fbim_status st = fbim_create(&p, out);
  if (st != FBIM_OK) return fail(c, st, "creating an RFD configuration failed");
  fbim_set_stream(*out, c->stream);
  for (auto &sh : c->shapes) {
    int32_t id = 0;
    st = fbim_add_shape(*out, sh.h.n_p, sh.h.ref_xy.data(), &id);
    if (st != FBIM_OK && st != FBIM_WACCURACY) return fail(c, st, fbim_last_error(*out));
  }
  return FBIM_OK;
}

}  // namespace

BatchEngine *engine_new() { return new BatchEngine(); }
void engine_delete(BatchEngine *E) { engine_destroy(E); }
const char *engine_error(const BatchEngine *E) { return E ? E->err.c_str() : ""; }
void engine_set_flags(BatchEngine *E, uint32_t flags) { E->flags = flags; }
void engine_set_stream(BatchEngine *E, hipStream_t s) {
  if (E->stream != s) destroy_graphs(E);
  E->stream = s;
  if (E->einfo) rocfft_execution_info_set_stream(E->einfo, s);
}

// Move every member to Q + dQ on the device; if one move is rejected (its
// context stays at Q), the members moved before it go back to Q as well.
fbim_status apply_moves(BatchEngine *E, const std::vector<fbim_ctx *> &mem, double *const *dQ) {
  for (size_t i = 0; i < mem.size(); ++i) {
    fbim_ctx *c = mem[i];
    const size_t n = c->n;
    EHIP(E, hipMemcpyAsync(c->d_qstep, c->d_q, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    EHIP(E, hipMemcpyAsync(c->d_thstep, c->d_theta, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    const fbim_status st = move_bodies(c, c->d_qstep, c->d_thstep, dQ[i], 1.0);
    if (st != FBIM_OK) {
      const std::string msg = c->err;
      for (size_t k = 0; k < i; ++k) move_bodies(mem[k], mem[k]->d_qstep, mem[k]->d_thstep, nullptr, 0.0);
      return efail(E, st, msg);
    }
  }
  return FBIM_OK;
}

// Batched EM-RFD solves of a list of systems: for member i, its RFD copies are
// rfd[0] (at Q + delta/2 Wt) and rfd[1] (at Q - delta/2 Wt).  U0 = N(Q) F +
// slip response and U+ = N(Q + delta/2 Wt) Wt of every member in one lockstep
// solve, then U- = N(Q - delta/2 Wt) Wt of every member in a second one that
// starts from U+.
fbim_status em_rfd_batch(BatchEngine *E, const std::vector<fbim_ctx *> &mem, double dt, double delta,
                         const double *const *F, const double *const *W_r, const double *const *W_grid,
                         const double *const *W_tilde, double *const *dQ, int32_t apply, fbim_info *info) {
  const int S = (int)mem.size();
  const bool rfd = delta > 0;  // delta = 0: no RFD term, U0 alone
  std::vector<fbim_info> inf(S);
  fbim_status worst = FBIM_OK;
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = mem[i];
    std::memset(&inf[i], 0, sizeof(fbim_info));
    // slip of the Brownian velocity (Lanczos + random field) into d_w
    fbim_status st = brownian_slip(c, dt, W_r[i], W_grid[i], c->d_w, &inf[i]);
    if (st != FBIM_OK && st != FBIM_ENOCONV) return efail(E, st, c->err);
    if (st != FBIM_OK) worst = st;
    for (int k = 0; rfd && k < 2; ++k) {
      if (!c->rfd[k]) {
        EST(clone_ctx(c, &c->rfd[k]));
      }
      fbim_ctx *r = c->rfd[k];
      r->stream = c->stream;
      r->p.tol_gmres = c->p.tol_rfd;  // the RFD solves stop at their own tolerance
      // the learned correction as the member uses it: its weights, refreshed at the
      // copy's configuration when the copy moves below
      r->mlp_on = false;
      if (c->mlp_on && c->mlp_init) {
        EST(ensure_mlp(r, c->n));
        EHIP(E, hipMemcpyAsync(r->d_mw, c->d_mw, FBIM_MLP_NPARAM * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        r->mlp_sym = c->mlp_sym;
        r->mlp_init = true;
        r->mlp_on = true;
      }
      if (!r->have_bodies || r->n != c->n || r->h_shape != c->h_shape) {
        // first use (or new bodies): the copy takes the member's bodies at the
        // configuration its caller last gave, then moves on the device
        st = fbim_set_bodies(r, c->n, c->h_shape.data(), c->h_q.data(), c->h_theta.data());
        if (st != FBIM_OK) return efail(E, st, fbim_last_error(r));
      }
      // Q +- delta/2 Wt, computed on the device from the member's configuration
      st = move_bodies(r, c->d_q, c->d_theta, W_tilde[i], k == 0 ? 0.5 * delta : -0.5 * delta);
      if (st != FBIM_OK) return efail(E, st, fbim_last_error(r));
    }
  }
  // one engine over members and their RFD copies
  E->sys.clear();
  for (auto *c : mem) E->sys.push_back(c);
  if (rfd) {
    for (auto *c : mem) E->sys.push_back(c->rfd[0]);
    for (auto *c : mem) E->sys.push_back(c->rfd[1]);
  }
  EST(engine_prepare(E));
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = mem[i];
    if (rhs_one(c, F[i], c->d_w) != FBIM_OK) return efail(E, FBIM_EDEVICE, c->err);
    for (int k = 0; rfd && k < 2; ++k)
      if (rhs_one(c->rfd[k], W_tilde[i], nullptr) != FBIM_OK) return efail(E, FBIM_EDEVICE, c->rfd[k]->err);
  }
  // U0 and U+ in one lockstep solve; then U- from U+ (same right-hand side,
  // configurations delta apart: the initial residual is O(delta))
  std::vector<int> first(rfd ? 2 * S : S), second(S);
  for (int i = 0; i < (int)first.size(); ++i) first[i] = i;
  for (int i = 0; i < S; ++i) second[i] = 2 * S + i;
  std::vector<int> its, sts, its2, sts2;
  std::vector<double> res, res2;
  EST(solve_b(E, first, its, res, sts));
  if (rfd) {
    for (int i = 0; i < S; ++i) {
      const fbim_ctx *p = mem[i]->rfd[0], *m = mem[i]->rfd[1];
      EHIP(E, hipMemcpyAsync(m->d_x2, p->d_x2, (2 * (size_t)p->N + 3 * (size_t)p->n) * sizeof(double),
                             hipMemcpyDeviceToDevice, E->stream));
    }
    EST(solve_b(E, second, its2, res2, sts2, true));
    its.insert(its.end(), its2.begin(), its2.end());
    res.insert(res.end(), res2.begin(), res2.end());
    sts.insert(sts.end(), sts2.begin(), sts2.end());
  }
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = mem[i];
    const size_t n3 = 3 * (size_t)c->n, twoN = 2 * (size_t)c->N;
    hipStream_t s = c->stream;
    EHIP(E, launch_axpby(n3, dt, c->d_x2 + twoN, 0.0, dQ[i], s));
    if (rfd) {
      const double *Up = c->rfd[0]->d_x2 + twoN, *Um = c->rfd[1]->d_x2 + twoN;
      EHIP(E, launch_axpby(n3, dt * c->p.kT / delta, Up, 1.0, dQ[i], s));
      EHIP(E, launch_axpby(n3, -dt * c->p.kT / delta, Um, 1.0, dQ[i], s));
    }
    for (int k = 0; k < (rfd ? 3 : 1); ++k) {
      const int j = i + k * S;
      inf[i].gmres_iters += its[j];
      inf[i].gmres_solves += 1;
      inf[i].gmres_residual = std::max(inf[i].gmres_residual, res[j]);
      if (sts[j] != FBIM_OK) worst = (fbim_status)sts[j];
    }
    inf[i].status = sts[i];
  }
  if (apply) EST(apply_moves(E, mem, dQ));
  EHIP(E, hipStreamSynchronize(E->stream));
  if (info)
    for (int i = 0; i < S; ++i) info[i] = inf[i];
  return worst;
}

// One AB2-RFD step of every member: the EM-RFD displacement (engine E, members
// left at Q), then N^n F^n of every member in one lockstep solve on engine Em
// (members only), dQ += dt/2 (N^n F^n - hist) and hist = N^n F^n.
fbim_status ab2_rfd_batch(BatchEngine *E, BatchEngine *Em, const std::vector<fbim_ctx *> &mem, double dt,
                          double delta, const double *const *F, const double *const *W_r,
                          const double *const *W_grid, const double *const *W_tilde, double *const *hist,
                          bool have_hist, double *const *dQ, int32_t apply, fbim_info *info) {
  const int S = (int)mem.size();
  std::vector<fbim_info> inf(S);
  fbim_status worst = em_rfd_batch(E, mem, dt, delta, F, W_r, W_grid, W_tilde, dQ, 0, inf.data());
  if (worst != FBIM_OK && worst != FBIM_ENOCONV) return worst;
  Em->sys = mem;
  fbim_status st = engine_prepare(Em);
  if (st != FBIM_OK) return efail(E, st, Em->err);
  for (int i = 0; i < S; ++i)
    if (rhs_one(mem[i], F[i], nullptr) != FBIM_OK) return efail(E, FBIM_EDEVICE, mem[i]->err);
  std::vector<int> all(S), its, sts;
  std::vector<double> res;
  for (int i = 0; i < S; ++i) all[i] = i;
  st = solve_b(Em, all, its, res, sts);
  if (st != FBIM_OK) return efail(E, st, Em->err);
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = mem[i];
    const size_t n3 = 3 * (size_t)c->n;
    hipStream_t s = c->stream;
    const double *NF = c->d_x2 + 2 * (size_t)c->N;
    if (have_hist) {
      EHIP(E, launch_axpby(n3, 0.5 * dt, NF, 1.0, dQ[i], s));
      EHIP(E, launch_axpby(n3, -0.5 * dt, hist[i], 1.0, dQ[i], s));
    }
    EHIP(E, hipMemcpyAsync(hist[i], NF, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    inf[i].gmres_iters += its[i];
    inf[i].gmres_solves += 1;
    inf[i].gmres_residual = std::max(inf[i].gmres_residual, res[i]);
    if (sts[i] != FBIM_OK) worst = (fbim_status)sts[i];
  }
  if (apply) EST(apply_moves(E, mem, dQ));
  EHIP(E, hipStreamSynchronize(E->stream));
  if (info)
    for (int i = 0; i < S; ++i) info[i] = inf[i];
  return worst;
}

}  // namespace fbim

struct fbim_batch {
  std::vector<fbim_ctx *> mem;
  fbim::BatchEngine *eng = nullptr, *rfd = nullptr;
  hipStream_t stream = nullptr;
  uint32_t flags = 0;
  std::string err;
};

namespace {
fbim_status bfail(fbim_batch *b, fbim_status s, const std::string &m) {
  if (b) b->err = m;
  return s;
}
// each member's noise: the caller's, or drawn by the member's generator (no W_tilde
// without the RFD term)
fbim_status batch_noise(fbim_batch *b, double delta, const double *const *W_r, const double *const *W_grid,
                        const double *const *W_tilde, std::vector<const double *> &wr,
                        std::vector<const double *> &wg, std::vector<const double *> &wt) {
  const size_t S = b->mem.size();
  wr.assign(S, nullptr);
  wg.assign(S, nullptr);
  wt.assign(S, nullptr);
  for (size_t i = 0; i < S; ++i) {
    wr[i] = W_r ? W_r[i] : nullptr;
    wg[i] = W_grid ? W_grid[i] : nullptr;
    wt[i] = W_tilde ? W_tilde[i] : nullptr;
    const fbim_status sn = fbim::fill_noise(b->mem[i], wr[i], wg[i], delta > 0 ? &wt[i] : nullptr);
    if (sn != FBIM_OK) return bfail(b, sn, b->mem[i]->err);
  }
  return FBIM_OK;
}

fbim_status from_engine(fbim_batch *b, fbim::BatchEngine *E, fbim_status s) {
  if (s != FBIM_OK) b->err = E->err;
  return s;
}
}  // namespace

extern "C" {

fbim_status fbim_batch_create(int32_t S, const fbim_params *params, fbim_batch **out) {
  if (S < 1 || !params || !out) return FBIM_EINVAL;
  *out = nullptr;
  for (int i = 1; i < S; ++i)
    if (params[i].precision != params[0].precision) return FBIM_EINVAL;
  auto *b = new fbim_batch();
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = nullptr;
    const fbim_status st = fbim_create(&params[i], &c);
    if (st != FBIM_OK) {
      fbim_batch_destroy(b);
      return st;
    }
    b->mem.push_back(c);
  }
  b->eng = fbim::engine_new();
  b->rfd = fbim::engine_new();
  *out = b;
  return FBIM_OK;
}

void fbim_batch_destroy(fbim_batch *b) {
  if (!b) return;
  fbim::engine_destroy(b->eng);
  fbim::engine_destroy(b->rfd);
  for (auto *c : b->mem) fbim_destroy(c);
  delete b;
}

const char *fbim_batch_last_error(const fbim_batch *b) { return b ? b->err.c_str() : "null batch"; }

fbim_ctx *fbim_batch_member(fbim_batch *b, int32_t s) {
  if (!b || s < 0 || s >= (int32_t)b->mem.size()) return nullptr;
  return b->mem[s];
}

fbim_status fbim_batch_set_stream(fbim_batch *b, void *stream) {
  if (!b) return FBIM_EINVAL;
  b->stream = (hipStream_t)stream;
  for (auto *c : b->mem) {
    const fbim_status st = fbim_set_stream(c, stream);
    if (st != FBIM_OK) return bfail(b, st, c->err);
  }
  fbim::engine_set_stream(b->eng, b->stream);
  fbim::engine_set_stream(b->rfd, b->stream);
  return FBIM_OK;
}

fbim_status fbim_batch_set_flags(fbim_batch *b, uint32_t flags) {
  if (!b || (flags & ~FBIM_BATCH_GRAPH)) return bfail(b, FBIM_EINVAL, "unknown batch flag");
  b->flags = b->eng->flags = b->rfd->flags = flags;
  return FBIM_OK;
}

fbim_status fbim_batch_apply_M(fbim_batch *b, const double *const *mu, double *const *out) {
  if (!b || !mu || !out) return bfail(b, FBIM_EINVAL, "null argument");
  fbim::BatchEngine *E = b->eng;
  E->sys = b->mem;
  fbim_status st = fbim::engine_prepare(E);
  if (st != FBIM_OK) return from_engine(b, E, st);
  const int S = (int)b->mem.size();
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = b->mem[i];
    if (hipMemcpyAsync(c->d_t1, mu[i], 2 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, E->stream) !=
        hipSuccess)
      return bfail(b, FBIM_EDEVICE, "copy of mu failed");
  }
  st = fbim::run_operator(E, E->full, E->mixed && b->mem[0]->cur32, false);
  if (st != FBIM_OK) return from_engine(b, E, st);
  for (int i = 0; i < S; ++i) {
    fbim_ctx *c = b->mem[i];
    if (hipMemcpyAsync(out[i], c->d_by, 2 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, E->stream) !=
        hipSuccess)
      return bfail(b, FBIM_EDEVICE, "copy of the result failed");
  }
  return FBIM_OK;
}

fbim_status fbim_batch_mobility(fbim_batch *b, const double *const *F, const double *const *slip, double *const *U,
                                fbim_info *info) {
  if (!b || !F || !U) return bfail(b, FBIM_EINVAL, "null argument");
  const double t0 = fbim::now_ms();
  fbim::BatchEngine *E = b->eng;
  E->sys = b->mem;
  fbim_status st = fbim::engine_prepare(E);
  if (st != FBIM_OK) return from_engine(b, E, st);
  const int S = (int)b->mem.size();
  for (int i = 0; i < S; ++i)
    if (fbim::rhs_one(b->mem[i], F[i], slip ? slip[i] : nullptr) != FBIM_OK)
      return bfail(b, FBIM_EDEVICE, b->mem[i]->err);
  std::vector<int> all(S), its, sts;
  std::vector<double> res;
  for (int i = 0; i < S; ++i) all[i] = i;
  st = fbim::solve_b(E, all, its, res, sts);
  if (st != FBIM_OK) return from_engine(b, E, st);
  fbim_status worst = FBIM_OK;
  for (int i = 0; i < S; ++i) {
    st = fbim::copy_out(E, b->mem[i], U[i]);
    if (st != FBIM_OK) return from_engine(b, E, st);
    if (sts[i] != FBIM_OK) worst = (fbim_status)sts[i];
  }
  if (hipStreamSynchronize(E->stream) != hipSuccess) return bfail(b, FBIM_EDEVICE, "stream synchronisation failed");
  if (info)
    for (int i = 0; i < S; ++i) {
      std::memset(&info[i], 0, sizeof(fbim_info));
      info[i].gmres_iters = its[i];
      info[i].gmres_solves = 1;
      info[i].gmres_residual = res[i];
      info[i].status = sts[i];
      info[i].ms_total = fbim::now_ms() - t0;
    }
  if (worst != FBIM_OK) b->err = "GMRES iteration limit reached in a batch system";
  return worst;
}

fbim_status fbim_batch_step_em_rfd(fbim_batch *b, double dt, double delta, const double *const *F,
                                   const double *const *W_r, const double *const *W_grid,
                                   const double *const *W_tilde, double *const *dQ, int32_t apply,
                                   fbim_info *info) {
  if (!b || !F || !dQ || !(dt > 0) || !(delta >= 0)) return bfail(b, FBIM_EINVAL, "invalid arguments");
  const double t0 = fbim::now_ms();
  std::vector<const double *> wr, wg, wt;
  const fbim_status sn = batch_noise(b, delta, W_r, W_grid, W_tilde, wr, wg, wt);
  if (sn != FBIM_OK) return sn;
  const fbim_status st =
      fbim::em_rfd_batch(b->rfd, b->mem, dt, delta, F, wr.data(), wg.data(), wt.data(), dQ, apply, info);
  if (info)
    for (size_t i = 0; i < b->mem.size(); ++i) info[i].ms_total = fbim::now_ms() - t0;
  if (st != FBIM_OK) b->err = b->rfd->err;
  return st;
}

fbim_status fbim_batch_step_ab2_rfd(fbim_batch *b, double dt, double delta, const double *const *F,
                                    const double *const *W_r, const double *const *W_grid,
                                    const double *const *W_tilde, double *const *NF_hist, int32_t have_hist,
                                    double *const *dQ, int32_t apply, fbim_info *info) {
  if (!b || !F || !dQ || !NF_hist || !(dt > 0) || !(delta >= 0)) return bfail(b, FBIM_EINVAL, "invalid arguments");
  for (size_t i = 0; i < b->mem.size(); ++i)
    if (!NF_hist[i] || !F[i] || !dQ[i]) return bfail(b, FBIM_EINVAL, "null member pointer");
  const double t0 = fbim::now_ms();
  std::vector<const double *> wr, wg, wt;
  const fbim_status sn = batch_noise(b, delta, W_r, W_grid, W_tilde, wr, wg, wt);
  if (sn != FBIM_OK) return sn;
  const fbim_status st = fbim::ab2_rfd_batch(b->rfd, b->eng, b->mem, dt, delta, F, wr.data(), wg.data(), wt.data(),
                                             NF_hist, have_hist != 0, dQ, apply, info);
  if (info)
    for (size_t i = 0; i < b->mem.size(); ++i) info[i].ms_total = fbim::now_ms() - t0;
  if (st != FBIM_OK) b->err = b->rfd->err;
  return st;
}

}  // extern "C"
