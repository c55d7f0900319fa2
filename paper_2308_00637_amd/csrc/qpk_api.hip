// Host side of libqpk: the C ABI of include/qpk.h.  Builds the device layouts
// once (qp_create), then drives the kernels of qpk_kernels.hip for each step
// of Algorithm 1 (Section 3.2).  Host code only launches kernels, reads back a
// few scalars per IPM iteration and polls one stop flag during PCG; all
// arithmetic of the method runs on the GPU (the host only turns the CG
// coefficients into the optional spectrum estimate).
#include "qpk_internal.h"
#include "../../include/qpk.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

using namespace qpk;

struct qp_handle_s {
  std::string err;
  hipStream_t st = nullptr;
  int n = 0, m = 0, me = 0, k = 0, p_rows = 0, h_kind = 0, prec = 0, vk = VK_F64;
  int nRP = 0;
  int64_t nnz_rp = 0, nnz_xs = 0;
  // operators (float64 always; *_lo: reduced-precision copies for the PCG matvec)
  int32_t *rp_rowptr = nullptr, *rp_col = nullptr;
  double* rp_val = nullptr;
  void* rp_lo = nullptr;
  int32_t *xs_rowptr = nullptr, *xs_seg1 = nullptr, *xs_seg2 = nullptr, *xs_col = nullptr;
  double* xs_val = nullptr;
  void* xs_lo = nullptr;
  double* U = nullptr;
  void* U_lo = nullptr;
  double *wd = nullptr, *h0 = nullptr, *Cm = nullptr, *b = nullptr, *c = nullptr, *c_eff = nullptr;
  double *lA = nullptr, *uA = nullptr, *lx = nullptr, *ux = nullptr, *pw = nullptr, *pd = nullptr;
  double* diagH = nullptr;
  double* diagH0 = nullptr;  // dense-H diagonal and h0: the part of diag(H) not derived on the device
  bool has_xs = false, has_ts = false;
  // iterate
  double *x = nullptr, *lam = nullptr, *s = nullptr;
  double mu = 1.0;
  // Mehrotra rule: the residuals' complementarity target while tau_on (else mu)
  double tau = 0.0;
  bool tau_on = false;
  double *dlam_aff = nullptr, *ds_aff = nullptr;   // the predictor's direction
  bool solved = false;
  bool res_valid = false, sys_valid = false;
  // work
  double *res = nullptr, *rhs = nullptr, *jdiag = nullptr, *dl = nullptr, *qdiag = nullptr;
  double *wA_mv = nullptr, *wA_res = nullptr, *wA_rhs = nullptr, *jw = nullptr;
  double *we_mv = nullptr, *we_res = nullptr, *we_rhs = nullptr, *te = nullptr, *g = nullptr, *u = nullptr;
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr, *tmp = nullptr;
  double* ones = nullptr;   // N ones: the "diagonal" of plain CG (pcg_options::no_precond)
  double* kap_sol = nullptr;  // solution of the plain CG run for ipm_options::log_kappa_plain
  double *dir = nullptr, *ds_w = nullptr;   // dir = [dx | dlam] (n + me + 2m + 2n)
  double* arhs = nullptr;                    // adjoint right-hand side
  double* valign = nullptr;                  // 16-byte aligned copy of a caller vector
  double *part = nullptr, *ts_part = nullptr, *sc = nullptr;
  int* fl = nullptr;
  double* hsc = nullptr;  // pinned host copy of sc
  int* hfl = nullptr;     // pinned host copy of fl
  int* hpoll = nullptr;   // pinned, 2 x F_COUNT: flag snapshots of the PCG poll
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  int lpr_r = 16, lpr_x = 64, g_r = 1, g_x = 1, g_vec = 1, g_ts = 1, ts_chunk = 1, g_n = 1, g_ra = 1;
  // LDS-staged blocked PCG matvec passes
  struct Chunked {
    bool on = false;
    int nrows = 0, ncols = 0, nchunk = 0, nwork = 0, lpr = 16, chunk_cols = kChunkCols, kv = kKvDefault;
    int xcd_map = 1;
    int32_t* work = nullptr;
    int32_t* rowptr = nullptr;
    uint16_t* col = nullptr;
    double* val = nullptr;
    void* val_lo = nullptr;
    double* partial = nullptr;
    int64_t nnz = 0;      // entries of the operator
    int64_t stored = 0;   // entries stored (segments padded to even length)
  } ck_r, ck_x;
  int g_rmv = 1, g_xmv = 1;             // partial counts of the PCG matvec passes
  int g_epi_r = 1, g_epi_x = 1;          // grids of the chunk epilogues
  bool alternate = true;                 // alternate the row direction of the blocked passes
  int64_t n_matvec = 0;                  // blocked K v products so far
  double* uw = nullptr;  // [u (p_rows) | wA (m)] for the PCG matvec
  // Blocked passes over P alone when every row of A repeats its own row of P:
  // twin[v] = the A row that repeats P row v, or -1
  bool fold_a = false;
  int32_t* twin = nullptr;
  // Fused single-read PCG product (H = P^T W P): the rows of the blocked row
  // side cut into two column halves, row ranges for block pairs
  struct Fused {
    bool on = false;
    bool failed = false;   // a pair's wait timed out once: two-pass from then on
    int nrows = 0, half = 0, nrange = 0;
    int32_t* range = nullptr;
    int32_t* rowinfo = nullptr;
    int32_t* rowptr = nullptr;
    uint16_t* col = nullptr;
    double* val = nullptr;
    void* val_lo = nullptr;
    int64_t stored = 0;
    double* xch = nullptr;
    double* ypart = nullptr;
    unsigned long long epoch = 0;
    int spin_max = 1 << 21;
  } fz;
  double* coef = nullptr;  // CG alpha/beta record (spectrum estimates), 2 * coef_cap
  int coef_cap = 0;
  std::vector<void*> allocs;
  // optional event timing of PCG launches
  struct Prof {
    bool on = false;
    int cap = 0;
    int every = 1;                               // time one dispatch in `every`
    std::vector<hipEvent_t> ev[QP_PROF_COUNT];  // 2 per timed dispatch
    int used[QP_PROF_COUNT] = {};
    int64_t seen[QP_PROF_COUNT] = {};            // dispatches offered so far
  } prof;
  // A chunk of PCG iterations captured as a HIP graph and replayed (float64
  // solves without profiling): the key holds what its kernels were built with.
  struct Graph {
    bool enabled = true;          // QPK_GRAPH=0: launch kernel by kernel
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;    // capture stream (the handle's may be the null stream)
    std::vector<uintptr_t> key;
    int64_t replays = 0, captures = 0;
  } gr;
  ~qp_handle_s() {
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (gr.graph) (void)hipGraphDestroy(gr.graph);
    if (gr.cap) (void)hipStreamDestroy(gr.cap);
    for (int c = 0; c < QP_PROF_COUNT; ++c)
      for (hipEvent_t e : prof.ev[c]) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
    if (hsc) (void)hipHostFree(hsc);
    if (hfl) (void)hipHostFree(hfl);
    if (hpoll) (void)hipHostFree(hpoll);
    for (hipEvent_t e : poll_ev)
      if (e) (void)hipEventDestroy(e);
  }
  int64_t N() const { return (int64_t)n + me + 2 * (int64_t)m; }
  int64_t nlam() const { return (int64_t)me + 2 * (int64_t)m + 2 * (int64_t)n; }
  int64_t ns() const { return 2 * (int64_t)m + 2 * (int64_t)n; }
  int64_t nres() const { return 5 * (int64_t)n + me + 4 * (int64_t)m; }
};

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      h->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return QP_ERR_HIP;                                                        \
    }                                                                           \
  } while (0)

#define CHK(expr)                      \
  do {                                 \
    qp_status s_ = (expr);             \
    if (s_ != QP_OK) return s_;        \
  } while (0)

static qp_status dalloc(qp_handle h, void** p, size_t bytes) {
  *p = nullptr;
  hipError_t e = hipMalloc(p, bytes ? bytes : 8);
  if (e != hipSuccess) {
    h->err = std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e);
    return QP_ERR_ALLOC;
  }
  h->allocs.push_back(*p);
  return QP_OK;
}

template <typename T>
static qp_status dalloc_t(qp_handle h, T** p, int64_t count) {
  return dalloc(h, reinterpret_cast<void**>(p), sizeof(T) * (size_t)std::max<int64_t>(count, 0));
}

template <typename T>
static qp_status upload(qp_handle h, T** p, const T* src, int64_t count) {
  CHK(dalloc_t(h, p, count));
  if (count > 0) HIPCHK(hipMemcpyAsync(*p, src, sizeof(T) * count, hipMemcpyHostToDevice, h->st));
  return QP_OK;
}

static inline uint16_t to_bf16(double v) {
  float f = (float)v;
  uint32_t bits;
  std::memcpy(&bits, &f, 4);
  if ((bits & 0x7f800000u) == 0x7f800000u) return (uint16_t)(bits >> 16);  // inf / nan
  const uint32_t rounding = 0x7fffu + ((bits >> 16) & 1u);                 // nearest even
  return (uint16_t)((bits + rounding) >> 16);
}

static qp_status upload_lo(qp_handle h, void** p, const std::vector<double>& v) {
  if (h->vk == VK_F32 || h->vk == VK_F32X) {
    std::vector<float> f(v.size());
    for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
    float* d;
    CHK(upload(h, &d, f.data(), (int64_t)f.size()));
    HIPCHK(hipStreamSynchronize(h->st));
    *p = d;
  } else {
    std::vector<uint16_t> f(v.size());
    for (size_t i = 0; i < v.size(); ++i) f[i] = to_bf16(v[i]);
    uint16_t* d;
    CHK(upload(h, &d, f.data(), (int64_t)f.size()));
    HIPCHK(hipStreamSynchronize(h->st));
    *p = d;
  }
  return QP_OK;
}

static int pow2_clamp(double v, int lo, int hi) {
  int p = lo;
  while (p < hi && p * 2 <= v) p *= 2;
  return p;
}

static int grid_cap(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ------------------------------------------------------------ arg builders
static VecArgs vec_args(qp_handle h) {
  VecArgs a{};
  a.n = h->n; a.m = h->m; a.me = h->me; a.N = (int32_t)h->N();
  a.x = h->x; a.lam = h->lam; a.s = h->s;
  a.lA = h->lA; a.uA = h->uA; a.lx = h->lx; a.ux = h->ux; a.b = h->b;
  a.mu = h->mu; a.res = h->res; a.rhs = h->rhs; a.jdiag = h->jdiag; a.dl = h->dl;
  a.wA = h->wA_rhs; a.jw = h->jw; a.we = h->we_rhs;
  a.dx = h->dir; a.dlam = h->dir + h->n; a.ds = h->ds_w; a.dlam_w = h->dir + h->n;
  a.gamma = 0.99; a.part = h->part; a.sc = h->sc; a.fl = h->fl;
  return a;
}

static RowArgs row_args(qp_handle h, bool lo) {
  RowArgs a{};
  a.p_rows = h->p_rows; a.m = h->m; a.n = h->n; a.me = h->me;
  a.rowptr = h->rp_rowptr; a.col = h->rp_col;
  a.val = lo ? h->rp_lo : (const void*)h->rp_val;
  a.w = h->pw; a.d = h->pd; a.u = h->u; a.lA = h->lA; a.uA = h->uA;
  a.lam = h->lam; a.s = h->s; a.mu = h->mu; a.res = h->res;
  a.tau = h->tau_on ? h->tau : h->mu;
  return a;
}

static ColArgs col_args(qp_handle h, bool lo) {
  ColArgs a{};
  a.n = h->n; a.me = h->me; a.m = h->m; a.p_rows = h->p_rows; a.k = h->k;
  a.rowptr = h->xs_rowptr; a.seg1 = h->xs_seg1; a.seg2 = h->xs_seg2; a.col = h->xs_col;
  a.val = h->has_xs ? (lo ? h->xs_lo : (const void*)h->xs_val) : nullptr;
  a.use_hx = 1; a.use_pt = 1; a.use_at = 1;
  a.U = lo ? h->U_lo : (const void*)h->U;
  a.g = h->g; a.Cm = h->Cm; a.qdiag = h->qdiag;
  a.c = h->c_eff; a.h0 = h->h0; a.lam = h->lam; a.s = h->s; a.lx = h->lx; a.ux = h->ux;
  a.mu = h->mu; a.diagH = h->diagH; a.wd = h->wd; a.w = h->pw;
  a.tau = h->tau_on ? h->tau : h->mu;
  return a;
}

static TsArgs ts_args(qp_handle h, bool lo, const double* v) {
  TsArgs a{};
  a.n = h->n; a.k = h->k; a.me = h->me;
  a.U = lo ? h->U_lo : (const void*)h->U;
  a.Cm = h->Cm; a.v = v; a.part = h->ts_part; a.chunk = h->ts_chunk;
  return a;
}

static TsFinishArgs tsf_args(qp_handle h) {
  TsFinishArgs a{};
  a.n = h->n; a.k = h->k; a.me = h->me; a.grid = h->g_ts;
  a.part = h->ts_part; a.wd = h->wd; a.g = h->g; a.te = h->te;
  a.b = h->b; a.lam = h->lam; a.mu = h->mu; a.res = h->res;
  return a;
}

// Event pair for the next dispatch of category c (null pair unless profiling
// is on and the category still has free slots).
static KEvents prof_slot(qp_handle h, int c, bool active) {
  KEvents e;
  if (!active || !h->prof.on) return e;
  if (h->prof.seen[c]++ % h->prof.every != 0 || h->prof.used[c] >= h->prof.cap) return e;
  const int slot = h->prof.used[c]++;
  e.start = h->prof.ev[c][2 * slot];
  e.stop = h->prof.ev[c][2 * slot + 1];
  return e;
}

// ---------------------------------------------------------------- steps
// Step a1: residual stack at (x, lam, s, mu) and its norms (into sc).
static qp_status run_residuals(qp_handle h) {
  if (h->has_ts) {
    HIPCHK(launch_ts_reduce(VK_F64, ts_args(h, false, h->x), h->g_ts, h->st));
    TsFinishArgs f = tsf_args(h);
    f.we = h->we_res;
    f.partout = h->part + P_NTS_RE * kGridMax;
    HIPCHK(launch_ts_finish(TS_RESID, f, h->st));
  }
  if (h->nRP > 0) {
    RowArgs a = row_args(h, false);
    a.r0 = 0; a.r1 = h->nRP; a.v = h->x; a.wA = h->wA_res; a.resw = h->res;
    a.part0 = h->part + P_NR_PRIMAL * kGridMax;
    a.part1 = h->part + P_NR_COMPL * kGridMax;
    HIPCHK(launch_rowpass(R_RESID, VK_F64, h->lpr_r, a, h->g_r, h->st));
  }
  ColArgs c = col_args(h, false);
  c.src_hx = h->x; c.src_pt = h->u; c.src_at = h->wA_res; c.we = h->we_res; c.v = h->x;
  c.res = h->res;
  c.part0 = h->part + P_NX_DUAL * kGridMax;
  c.part1 = h->part + P_NX_PRIMAL * kGridMax;
  c.part2 = h->part + P_NX_COMPL * kGridMax;
  HIPCHK(launch_colpass(X_RESID, VK_F64, h->lpr_x, c, h->g_x, h->st));
  HIPCHK(launch_finish_norms(vec_args(h), h->nRP > 0 ? h->g_r : 0, h->g_x, h->st));
  h->res_valid = true;
  return QP_OK;
}

// Steps a2, a3: D, the eq. (9) right-hand side, diag(K), Q's diagonal.
static qp_status run_system(qp_handle h) {
  if (!h->res_valid) CHK(run_residuals(h));
  VecArgs v = vec_args(h);
  HIPCHK(launch_rhs_lam(v, h->st));
  ColArgs c = col_args(h, false);
  c.use_hx = 0; c.use_pt = 0; c.use_at = 1;
  c.src_at = h->wA_rhs; c.src_at2 = h->jw; c.we = h->we_rhs;
  c.res_in = h->res; c.rhs = h->rhs; c.jdiag = h->jdiag; c.qdiag_out = h->qdiag;
  HIPCHK(launch_colpass(X_RHS, VK_F64, h->lpr_x, c, h->g_x, h->st));
  h->sys_valid = true;
  return QP_OK;
}

static qp_status prepare(qp_handle h) {
  if (!h->sys_valid) CHK(run_system(h));
  return QP_OK;
}

static ChunkArgs chunk_args(const qp_handle_s::Chunked& k, bool lo, const double* src, bool reverse) {
  ChunkArgs c{};
  c.reverse = reverse ? 1 : 0;
  c.xcd_map = k.xcd_map;
  c.nrows = k.nrows; c.ncols = k.ncols; c.nchunk = k.nchunk; c.chunk_cols = k.chunk_cols;
  c.work = k.work; c.rowptr = k.rowptr; c.col = k.col;
  c.val = lo ? k.val_lo : (const void*)k.val;
  c.src = src; c.partial = k.partial;
  c.kv = k.kv;
  c.nstored = (int32_t)k.stored;
  return c;
}

// True when a PCG product leaves the column epilogue to k_cg_update: the
// column side has several chunks (so an epilogue), and the single-chunk row
// pass can form all of p.q from its row terms and a slice of the diagonal.
static bool pcg_fuses_epilogue(qp_handle h) {
  return h->ck_x.on && h->ck_x.nchunk > 1 && h->ck_r.on && h->ck_r.nchunk == 1 && h->nRP > 0;
}

static bool fused_active(qp_handle h) { return h->fz.on && !h->fz.failed; }

// Step a4: y = K v (v, y: K-vectors).  lo selects the reduced-precision
// operator copies.  With the fused layout active, one pass over the rows forms
// the lam-part and per-range x-parts (k_fused); a PCG iteration's update sums
// the x-parts itself, other products through the column epilogue.  done/bump: PCG early exit and iteration counter.  fuse
// (PCG iterations only, when pcg_fuses_epilogue): the x-part of y is left as
// per-chunk partials, and the row pass's partials carry all of p.q.
static qp_status run_matvec(qp_handle h, bool lo, const double* v, double* y, const int* done,
                            int* bump, bool fuse = false, int parity = -1) {
  const int vk = lo ? h->vk : VK_F64;
  const bool prof = bump != nullptr;  // only the PCG iteration's own matvec is timed
  // row direction of the blocked passes: by the PCG iteration's parity when
  // given (the same in a replayed chunk as in launches one by one), else by
  // the count of products
  const bool rev = h->alternate && ((parity >= 0 ? parity : h->n_matvec++) & 1);
  if (reinterpret_cast<uintptr_t>(v) & 15) {
    // the blocked row pass stages v with 16-byte loads
    HIPCHK(launch_copy(v, h->valign, h->N(), 1.0, h->st));
    v = h->valign;
  }
  if (h->has_ts) {
    TsArgs t = ts_args(h, lo, v);
    t.done = done;
    const KEvents ev = prof_slot(h, QP_PROF_TSREDUCE, prof);
    HIPCHK(launch_ts_reduce(vk, t, h->g_ts, h->st, &ev));
    TsFinishArgs f = tsf_args(h);
    f.we = h->we_mv; f.vl = v + h->n; f.yl = y + h->n;
    f.partout = h->part + P_DOT_TS * kGridMax; f.done = done;
    HIPCHK(launch_ts_finish(TS_MATVEC, f, h->st));
  }
  if (fused_active(h)) {
    RowArgs a = row_args(h, lo);
    a.r0 = 0; a.r1 = h->fz.nrows; a.v = v;
    a.vl = h->m > 0 ? v + h->n : v;
    a.dl = h->dl; a.yl = y + h->n;
    a.wA = h->wA_mv; a.part0 = h->part + P_DOT_R * kGridMax; a.done = done; a.bump = bump;
    if (h->fold_a) a.twin = h->twin;
    a.xdot = fuse ? 1 : 0;
    a.qdiag = h->qdiag;
    a.Cm = h->Cm;
    a.we = h->we_mv;
    FusedArgs f{};
    f.nrows = h->fz.nrows; f.ncols = h->n; f.half = h->fz.half; f.nrange = h->fz.nrange;
    f.range = h->fz.range; f.rowptr = h->fz.rowptr; f.col = h->fz.col;
    f.val = lo ? h->fz.val_lo : (const void*)h->fz.val;
    f.nstored = (int32_t)h->fz.stored;
    f.src = v; f.rowinfo = h->fz.rowinfo; f.xch = h->fz.xch; f.abort = h->fl + F_FUSEFAIL;
    f.epoch = ++h->fz.epoch; f.spin_max = h->fz.spin_max; f.ypart = h->fz.ypart;
    const KEvents ev = prof_slot(h, QP_PROF_FUSED, prof);
    HIPCHK(launch_fused(vk, f, a, h->st, &ev));
    if (!fuse) {
      ChunkArgs ca{};
      ca.nrows = h->n; ca.ncols = h->n; ca.nchunk = h->fz.nrange; ca.partial = h->fz.ypart;
      ColArgs c = col_args(h, lo);
      c.we = h->we_mv; c.v = v; c.y = y;
      c.part0 = h->part + P_DOT_X * kGridMax; c.done = done;
      HIPCHK(launch_chunk_epilogue_col(ca, c, h->g_epi_x, h->st));
    }
    return QP_OK;
  }
  if (h->nRP > 0) {
    RowArgs a = row_args(h, lo);
    // the lam-part pointers are only dereferenced for rows of A; without them
    // (m == 0) they point at valid memory for the blocked pass's clamped loads
    a.r0 = 0; a.r1 = h->nRP; a.v = v;
    a.vl = h->m > 0 ? v + h->n : v;
    a.dl = h->dl; a.yl = y + h->n;
    a.wA = h->wA_mv; a.part0 = h->part + P_DOT_R * kGridMax; a.done = done;
    if (h->fold_a) a.twin = h->twin;
    if (fuse && pcg_fuses_epilogue(h)) {
      a.xdot = 1;
      a.qdiag = h->qdiag;
      a.Cm = h->Cm;
      a.we = h->we_mv;
    }
    const KEvents ev = prof_slot(h, QP_PROF_ROWPASS, prof);
    if (h->ck_r.on) {
      ChunkArgs ca = chunk_args(h->ck_r, lo, v, rev);
      if (h->ck_r.nchunk == 1) {
        HIPCHK(launch_chunked(CE_ROW, vk, h->ck_r.lpr, ca, a, ColArgs{}, h->ck_r.nwork, h->st, &ev));
      } else {
        HIPCHK(launch_chunked(CE_PARTIAL, vk, h->ck_r.lpr, ca, a, ColArgs{}, h->ck_r.nwork, h->st,
                              &ev));
        const KEvents ee = prof_slot(h, QP_PROF_EPILOGUE, prof);
        HIPCHK(launch_chunk_epilogue_row(ca, a, h->g_epi_r, h->st, &ee));
      }
    } else {
      HIPCHK(launch_rowpass(R_MATVEC, vk, h->lpr_r, a, h->g_rmv, h->st, &ev));
    }
  }
  ColArgs c = col_args(h, lo);
  c.src_hx = v; c.src_pt = h->u; c.src_at = h->wA_mv; c.we = h->we_mv; c.v = v; c.y = y;
  c.part0 = h->part + P_DOT_X * kGridMax; c.done = done; c.bump = bump;
  const KEvents ev = prof_slot(h, QP_PROF_COLPASS, prof);
  if (h->ck_x.on) {
    ChunkArgs ca = chunk_args(h->ck_x, lo, h->uw, rev);
    if (h->ck_x.nchunk == 1) {
      HIPCHK(launch_chunked(CE_COL, vk, h->ck_x.lpr, ca, RowArgs{}, c, h->ck_x.nwork, h->st, &ev));
    } else if (fuse && pcg_fuses_epilogue(h)) {
      HIPCHK(launch_chunked(CE_PARTIAL, vk, h->ck_x.lpr, ca, RowArgs{}, c, h->ck_x.nwork, h->st,
                            &ev));
    } else {
      ColArgs c0 = c;
      c0.bump = nullptr;
      HIPCHK(launch_chunked(CE_PARTIAL, vk, h->ck_x.lpr, ca, RowArgs{}, c0, h->ck_x.nwork, h->st,
                            &ev));
      const KEvents ee = prof_slot(h, QP_PROF_EPILOGUE, prof);
      HIPCHK(launch_chunk_epilogue_col(ca, c, h->g_epi_x, h->st, &ee));
    }
  } else {
    HIPCHK(launch_colpass(X_MATVEC, vk, h->lpr_x, c, h->g_xmv, h->st, &ev));
  }
  return QP_OK;
}

static CgArgs cg_args(qp_handle h, const double* rhs, double* sol, const pcg_options& o) {
  CgArgs a{};
  a.N = (int32_t)h->N(); a.n = h->n;
  a.x = sol; a.r = h->cg_r; a.z = h->cg_z; a.p = h->cg_p; a.q = h->cg_q;
  a.rhs = rhs; a.jdiag = h->jdiag; a.part = h->part; a.fl = h->fl; a.sc = h->sc;
  a.g_vec = h->g_vec; a.g_r = h->nRP > 0 ? h->g_rmv : 0; a.g_x = h->g_xmv; a.has_ts = h->has_ts;
  a.me = h->me;
  a.tol = o.tol; a.maxit = o.maxit;
  return a;
}

static qp_status read_back(qp_handle h) {
  HIPCHK(hipMemcpyAsync(h->hsc, h->sc, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipMemcpyAsync(h->hfl, h->fl, sizeof(int) * F_COUNT, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

// Extreme eigenvalues of the symmetric tridiagonal matrix (diagonal d, off-
// diagonal e, size k) by Sturm-sequence bisection.
static void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e,
                             double* lo_out, double* hi_out) {
  const int k = (int)d.size();
  double lo = INFINITY, hi = -INFINITY;
  for (int j = 0; j < k; ++j) {
    const double r = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < k ? std::fabs(e[j]) : 0.0);
    lo = std::min(lo, d[j] - r);
    hi = std::max(hi, d[j] + r);
  }
  // number of eigenvalues below x
  auto below = [&](double x) {
    int cnt = 0;
    double q = 1.0;
    for (int j = 0; j < k; ++j) {
      q = d[j] - x - (j > 0 ? e[j - 1] * e[j - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int want) {   // smallest x with below(x) >= want
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 1e-14 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double mid = 0.5 * (a + b);
      if (below(mid) >= want) b = mid;
      else a = mid;
    }
    return 0.5 * (a + b);
  };
  *lo_out = kth(1);
  *hi_out = kth(k);
}

// Step a5: Jacobi PCG (needs prepare()).  Also reports the true relative
// residual ||rhs - K sol|| / ||rhs|| with the float64 operator.
static qp_status true_residual(qp_handle h, const double* rhs, const double* sol) {
  CHK(run_matvec(h, false, sol, h->tmp, nullptr, nullptr));
  HIPCHK(launch_sqdiff(rhs, h->tmp, h->N(), h->part + P_CHK * kGridMax, h->g_vec, h->st));
  HIPCHK(launch_finish_sum(h->part + P_CHK * kGridMax, h->g_vec, h->sc + S_RELRES, h->st));
  return QP_OK;
}

static qp_status run_pcg(qp_handle h, const double* rhs, double* sol, const pcg_options& o,
                         pcg_info* info, bool force64 = false) {
  CgArgs a = cg_args(h, rhs, sol, o);
  if (o.no_precond) {
    if (!h->ones) {
      CHK(dalloc_t(h, &h->ones, h->N()));
      HIPCHK(launch_fill(h->ones, h->N(), 1.0, h->st));
    }
    a.jdiag = h->ones;
  }
  HIPCHK(launch_cg_init(a, h->st));
  const bool fused = fused_active(h);
  const bool fuse = fused || pcg_fuses_epilogue(h);
  CgArgs au = a;   // k_cg_update's view: q's x-part from the column or range partials
  if (fuse) {
    au.qpart = fused ? h->fz.ypart : h->ck_x.partial;
    au.nchunk = fused ? h->fz.nrange : h->ck_x.nchunk;
    if (fused) au.g_r = 2 * h->fz.nrange;
    au.g_x = 0;   // p.q is all in the row pass's partials
    au.me = h->me;
    au.qdiag = h->qdiag;
    au.Cm = h->Cm;
    au.we = h->we_mv;
  }
  const bool lo = h->vk != VK_F64 && !force64;
  // CG coefficients for the spectrum estimate (float64 solves: no restarts)
  const bool spectrum = o.spectrum != 0 && !lo;
  if (spectrum) {
    if (h->coef_cap < o.maxit) {
      if (h->coef) {
        (void)hipFree(h->coef);
        auto it = std::find(h->allocs.begin(), h->allocs.end(), (void*)h->coef);
        if (it != h->allocs.end()) h->allocs.erase(it);
        h->coef = nullptr;
      }
      CHK(dalloc_t(h, &h->coef, 2 * (int64_t)o.maxit));
      h->coef_cap = o.maxit;
    }
    a.coef = h->coef;
    au.coef = h->coef;
  }
  const int check = std::max(1, o.check_every);
  // One iteration's launches (product, update, direction update): queued
  // directly or recorded into the chunk graph.
  auto queue_iteration = [&](int iter) -> qp_status {
    CHK(run_matvec(h, lo, h->cg_p, h->cg_q, h->fl + F_DONE, h->fl + F_CNT, fuse, iter));
    const KEvents e1 = prof_slot(h, QP_PROF_CGUPDATE, true);
    HIPCHK(launch_cg_update(au, h->st, &e1));
    const KEvents e2 = prof_slot(h, QP_PROF_CGPUPDATE, true);
    HIPCHK(launch_cg_pupdate(a, h->st, &e2));
    return QP_OK;
  };
  // Chunks of `check` iterations replay one captured graph: the kernels'
  // arguments do not change from one chunk to the next (the fused pass's
  // exchange parity alternates within the chunk, `check` even), and every
  // kernel reads the stop flag itself.  Reduced-precision solves (residual
  // replacement between iterations) and profiled solves launch directly.
  const bool graph = h->gr.enabled && !lo && !h->prof.on && check >= 2 && (check % 2) == 0 &&
                     o.maxit >= check;
  if (graph) {
    // everything a captured kernel takes by value: pointers, options and mu
    // (the equality rows' penalty of the product)
    uint64_t mu_bits = 0, tol_bits = 0;
    std::memcpy(&mu_bits, &h->mu, sizeof(double));
    std::memcpy(&tol_bits, &o.tol, sizeof(double));
    const std::vector<uintptr_t> key = {
        (uintptr_t)rhs, (uintptr_t)sol, (uintptr_t)a.jdiag, (uintptr_t)au.coef, (uintptr_t)check,
        (uintptr_t)fused, (uintptr_t)fuse, (uintptr_t)tol_bits, (uintptr_t)mu_bits,
        (uintptr_t)o.maxit, (uintptr_t)h->fz.failed, (uintptr_t)h->alternate};
    if (!h->gr.exec || h->gr.key != key) {
      if (h->gr.exec) { (void)hipGraphExecDestroy(h->gr.exec); h->gr.exec = nullptr; }
      if (h->gr.graph) { (void)hipGraphDestroy(h->gr.graph); h->gr.graph = nullptr; }
      if (!h->gr.cap) HIPCHK(hipStreamCreateWithFlags(&h->gr.cap, hipStreamNonBlocking));
      // the launches are recorded on a stream of the handle's own (capture
      // is not allowed on the null stream); the graph then runs on h->st
      const hipStream_t user = h->st;
      h->st = h->gr.cap;
      hipError_t ec = hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal);
      qp_status cs = QP_OK;
      if (ec == hipSuccess)
        for (int c = 0; c < check && cs == QP_OK; ++c) cs = queue_iteration(c);
      hipGraph_t g = nullptr;
      if (ec == hipSuccess) ec = hipStreamEndCapture(h->st, &g);
      h->st = user;
      if (cs != QP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return cs;
      }
      HIPCHK(ec);
      h->gr.graph = g;
      HIPCHK(hipGraphInstantiate(&h->gr.exec, g, nullptr, nullptr, 0));
      h->gr.key = key;
      h->gr.captures++;
    }
  }
  int it = 0;
  CHK(read_back(h));
  bool done = h->hfl[F_DONE] != 0;
  const double rhsn = h->hsc[S_RHSNORM];
  while (it < o.maxit) {
    // The stop flag is polled one chunk late: chunk c is queued before the
    // host waits for chunk c-1's flags, so the GPU never drains while the host
    // reads them.  Iterations queued past convergence exit at once.
    int slot = 0;
    bool queued = false;
    while (!done && it < o.maxit) {
      const int chunk = std::min(check, o.maxit - it);
      if (graph && chunk == check) {
        HIPCHK(hipGraphLaunch(h->gr.exec, h->st));
        h->gr.replays++;
        it += chunk;
      } else for (int c = 0; c < chunk; ++c, ++it) {
        if (lo && o.rr_period > 0 && it > 0 && it % o.rr_period == 0) {
          // residual replacement: r = rhs - K x with the float64 operator
          CHK(run_matvec(h, false, sol, h->tmp, h->fl + F_DONE, nullptr));
          HIPCHK(launch_cg_restart(a, h->tmp, 0, h->st));
        }
        CHK(queue_iteration(it));
      }
      int* snap = h->hpoll + slot * F_COUNT;
      HIPCHK(hipMemcpyAsync(snap, h->fl, sizeof(int) * F_COUNT, hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipEventRecord(h->poll_ev[slot], h->st));
      if (queued) {
        HIPCHK(hipEventSynchronize(h->poll_ev[slot ^ 1]));
        done = h->hpoll[(slot ^ 1) * F_COUNT + F_DONE] != 0;
      }
      queued = true;
      slot ^= 1;
    }
    CHK(read_back(h));   // flags after everything queued
    done = h->hfl[F_DONE] != 0;
    if (!lo || h->hfl[F_STATUS] != 1) break;
    // Reduced-precision operator: the stop test saw the recurrence residual;
    // accept only if the float64 residual passes too, else restart from it.
    CHK(true_residual(h, rhs, sol));
    CHK(read_back(h));
    if (std::sqrt(h->hsc[S_RELRES]) <= o.tol * rhsn || h->hfl[F_ITERS] >= o.maxit) break;
    HIPCHK(launch_cg_restart(a, h->tmp, 1, h->st));
    it = h->hfl[F_ITERS];
    done = false;
  }
  // true residual with the float64 operator
  CHK(true_residual(h, rhs, sol));
  CHK(read_back(h));
  if (fused && h->hfl[F_FUSEFAIL]) {
    // a block pair of the fused product timed out waiting for its partner
    // (it never ran alongside): the products since are invalid.  Redo the
    // solve with the two-pass kernels, which need no partner.
    h->fz.failed = true;
    return run_pcg(h, rhs, sol, o, info, force64);
  }
  const int status = h->hfl[F_STATUS];
  pcg_info inf{};
  inf.iterations = h->hfl[F_ITERS];
  inf.converged = status == 1;
  inf.rhs_norm = h->hsc[S_RHSNORM];
  inf.status = QP_OK;
  if (status == QP_ERR_NOT_SPD_CODE) inf.status = QP_ERR_NOT_SPD;
  if (status == QP_ERR_NUMERIC_CODE) inf.status = QP_ERR_NUMERIC;
  if (status == 0) inf.iterations = o.maxit;
  inf.rel_residual = inf.rhs_norm > 0.0 ? std::sqrt(h->hsc[S_RELRES]) / inf.rhs_norm : 0.0;
  if (spectrum && status != 0 && inf.iterations > 0 && inf.status == QP_OK) {
    // Lanczos matrix of the preconditioned CG: d_j = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    // e_j = sqrt(beta_j)/alpha_j
    const int k = inf.iterations;
    std::vector<double> ab(2 * (size_t)k);
    HIPCHK(hipMemcpy(ab.data(), h->coef, sizeof(double) * 2 * k, hipMemcpyDeviceToHost));
    std::vector<double> d(k), e(k > 1 ? k - 1 : 0);
    for (int j = 0; j < k; ++j) {
      d[j] = 1.0 / ab[2 * j] + (j > 0 ? ab[2 * j - 1] / ab[2 * (j - 1)] : 0.0);
      if (j + 1 < k) e[j] = std::sqrt(ab[2 * j + 1]) / ab[2 * j];
    }
    tridiag_extremes(d, e, &inf.lambda_min, &inf.lambda_max);
  }
  bool escalate = false;
  if (lo) {
    if (inf.status != QP_OK || (inf.converged && !(inf.rel_residual <= o.tol))) {
      escalate = true;   // breakdown, or a converged recurrence the operator cannot honour
    } else if (!inf.converged) {
      // Stopped at the iteration cap, as float64 solves of hard systems do too
      // (the method then goes on with the iterate).  Redo it in float64 only
      // when the reduced operator, not the iteration budget, limited it: its
      // float64 residual well above the recurrence residual the PCG reached.
      HIPCHK(launch_finish_sum(h->part + P_RR * kGridMax, h->g_vec, h->sc + S_RECUR, h->st));
      CHK(read_back(h));
      const double recur = inf.rhs_norm > 0.0 ? std::sqrt(h->hsc[S_RECUR]) / inf.rhs_norm : 0.0;
      escalate = !(inf.rel_residual <= 10.0 * recur);
    }
  }
  if (escalate) {
    // the reduced-precision operator could not deliver this solve: redo it in float64
    pcg_info again{};
    const qp_status s2 = run_pcg(h, rhs, sol, o, &again, true);
    again.iterations += inf.iterations;
    again.escalated = 1;
    if (info) *info = again;
    return s2;
  }
  if (info) *info = inf;
  if (inf.status == QP_ERR_NOT_SPD) {
    h->err = "PCG met a non-positive curvature p^T K p (H not convex, or the iterate is broken)";
    return QP_ERR_NOT_SPD;
  }
  if (inf.status == QP_ERR_NUMERIC) {
    h->err = "PCG met a NaN or Inf";
    return QP_ERR_NUMERIC;
  }
  return QP_OK;
}

// Step a6: recovery of ds and the bound multipliers' steps, and the ratio
// test of step a7 (alphas into sc).
static qp_status run_recover(qp_handle h, double gamma) {
  if (h->m > 0) {
    RowArgs a = row_args(h, false);
    a.r0 = h->p_rows; a.r1 = h->nRP; a.v = h->dir; a.dlam = h->dir + h->n; a.ds = h->ds_w;
    a.part0 = h->part + P_MIN_S_R * kGridMax; a.part1 = h->part + P_MIN_L_R * kGridMax;
    HIPCHK(launch_rowpass(R_RECOVER, VK_F64, h->lpr_r, a, h->g_ra, h->st));
  }
  VecArgs v = vec_args(h);
  v.gamma = gamma;
  HIPCHK(launch_recover_x(v, h->g_n, h->st));
  HIPCHK(launch_finish_ratio(v, h->m > 0 ? h->g_ra : 0, h->g_n, h->st));
  return QP_OK;
}

static qp_status run_objective(qp_handle h, double* out) {
  if (h->p_rows > 0) {
    RowArgs a = row_args(h, false);
    a.r0 = 0; a.r1 = h->p_rows; a.v = h->x;
    HIPCHK(launch_rowpass(R_PU, VK_F64, h->lpr_r, a, h->g_r, h->st));
  }
  if (h->k > 0) {
    HIPCHK(launch_ts_reduce(VK_F64, ts_args(h, false, h->x), h->g_ts, h->st));
    TsFinishArgs f = tsf_args(h);
    f.we = h->we_mv;
    HIPCHK(launch_ts_finish(TS_GONLY, f, h->st));
  }
  ColArgs c = col_args(h, false);
  c.use_at = 0; c.src_hx = h->x; c.src_pt = h->u; c.v = h->x; c.part0 = h->part + P_OBJ * kGridMax;
  HIPCHK(launch_colpass(X_OBJ, VK_F64, h->lpr_x, c, h->g_x, h->st));
  HIPCHK(launch_finish_sum(h->part + P_OBJ * kGridMax, h->g_x, h->sc + S_OBJ, h->st));
  CHK(read_back(h));
  *out = h->hsc[S_OBJ];
  return QP_OK;
}

// Constant parts: diag(H) = diagH0 + diag(P^T W P) + sum_l wd_l U_jl^2 and
// c_eff = c - P^T W d.
static qp_status derive_constants(qp_handle h) {
  if (h->p_rows > 0 || h->k > 0) {
    ColArgs c = col_args(h, false);
    c.use_hx = 0; c.use_at = 0; c.use_pt = h->p_rows > 0;
    c.v = h->diagH0; c.y = h->diagH;
    HIPCHK(launch_colpass(X_DIAGH, VK_F64, h->lpr_x, c, h->g_x, h->st));
  } else {
    HIPCHK(launch_copy(h->diagH0, h->diagH, h->n, 1.0, h->st));
  }
  if (h->p_rows > 0 && h->pd) {
    ColArgs c = col_args(h, false);
    c.use_hx = 0; c.use_at = 0; c.use_pt = 1; c.src_pt = h->pd; c.c = h->c; c.y = h->c_eff;
    HIPCHK(launch_colpass(X_CEFF, VK_F64, h->lpr_x, c, h->g_x, h->st));
  } else {
    HIPCHK(launch_copy(h->c, h->c_eff, h->n, 1.0, h->st));
  }
  return QP_OK;
}

static qp_status run_init_state(qp_handle h, double mu) {
  h->mu = mu;
  VecArgs v = vec_args(h);
  HIPCHK(launch_init_x(v, grid_cap(std::max(h->n, h->me), kBlock, kGridMax), h->st));
  if (h->m > 0) {
    RowArgs a = row_args(h, false);
    a.r0 = h->p_rows; a.r1 = h->nRP; a.v = h->x; a.ds = h->s; a.yl = h->lam;
    HIPCHK(launch_rowpass(R_INIT, VK_F64, h->lpr_r, a, h->g_ra, h->st));
  }
  h->res_valid = h->sys_valid = false;
  h->solved = false;
  return QP_OK;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

void qp_default_pcg_options(pcg_options* o) {
  if (!o) return;
  o->tol = 1e-7;
  o->maxit = 5000;
  o->check_every = 8;
  o->rr_period = 0;
  o->spectrum = 0;
  o->no_precond = 0;
}

void qp_default_ipm_options(ipm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->gamma = 0.99;
  o->mu0 = 1.0;
  o->mu_tol = 1e-6;
  o->mu_div = 10.0;
  o->max_iter = 200;
  o->warm_start = 0;
  qp_default_pcg_options(&o->pcg);
}

const char* qp_status_string(int32_t s) {
  switch (s) {
    case QP_OK: return "ok";
    case QP_ERR_ARG: return "invalid argument";
    case QP_ERR_ALLOC: return "allocation failed";
    case QP_ERR_HIP: return "HIP runtime error";
    case QP_ERR_NOT_SPD: return "KKT matrix not positive definite";
    case QP_ERR_NUMERIC: return "NaN or Inf encountered";
    case QP_ERR_STATE: return "call not valid in the current state";
    case QP_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

static thread_local std::string g_create_error;

const char* qp_last_error(qp_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

// Split a CSR operator (sorted columns in [0, ncols)) into column chunks of
// kChunkCols with uint16 in-chunk offsets, stored chunk-major, and cut each
// chunk's rows into work items of about equal entry counts so that all items
// fit one wave of blocks (one block per CU, 256 CUs).
// Pairs every row of A with a row of P holding the same columns and values
// (bit for bit), each P row serving at most one A row.  Returns false, with
// twin untouched, unless every row of A finds one.
static bool match_twins(int64_t p_rows, const std::vector<int64_t>& prp, const int32_t* pcol,
                        const double* pval, int64_t m, const std::vector<int64_t>& arp,
                        const std::vector<int32_t>& acol, const std::vector<double>& aval,
                        std::vector<int32_t>& twin) {
  auto row_hash = [](const int32_t* c, const double* v, int64_t len) {
    uint64_t x = 1469598103934665603ull ^ (uint64_t)len;
    for (int64_t q = 0; q < len; ++q) {
      uint64_t b;
      std::memcpy(&b, &v[q], 8);
      x = (x ^ (uint64_t)(uint32_t)c[q]) * 1099511628211ull;
      x = (x ^ b) * 1099511628211ull;
    }
    return x;
  };
  std::unordered_multimap<uint64_t, int64_t> byhash;
  byhash.reserve((size_t)p_rows);
  for (int64_t v = 0; v < p_rows; ++v)
    byhash.emplace(row_hash(pcol + prp[v], pval + prp[v], prp[v + 1] - prp[v]), v);
  std::vector<int32_t> t((size_t)p_rows, -1);
  for (int64_t i = 0; i < m; ++i) {
    const int64_t len = arp[i + 1] - arp[i];
    const int32_t* c = acol.data() + arp[i];
    const double* v = aval.data() + arp[i];
    auto range = byhash.equal_range(row_hash(c, v, len));
    int64_t found = -1;
    for (auto it = range.first; it != range.second && found < 0; ++it) {
      const int64_t r = it->second;
      if (t[(size_t)r] >= 0 || prp[r + 1] - prp[r] != len) continue;
      if (std::memcmp(pcol + prp[r], c, 4 * (size_t)len) == 0 &&
          std::memcmp(pval + prp[r], v, 8 * (size_t)len) == 0)
        found = r;
    }
    if (found < 0) return false;
    t[(size_t)found] = (int32_t)i;
  }
  twin.swap(t);
  return true;
}

// Chunk-major storage of a CSR operator whose columns are cut into chunks of
// cw: chunk c holds its own CSR (row pointers c * (nrows + 1) ...) with uint16
// column offsets within the chunk; every (chunk, row) segment is padded with
// zero entries to even length, so kernels load entries in aligned pairs.
struct ChunkStore {
  int nchunk = 0;
  int64_t stored = 0;
  std::vector<int32_t> rowptr;
  std::vector<int64_t> nnz;      // entries per chunk, with the padding
  std::vector<uint16_t> col;
  std::vector<double> val;
};

static qp_status chunk_store(qp_handle h, const std::vector<int32_t>& rp, const std::vector<int32_t>& col,
                             const std::vector<double>& val, int ncols, int cw, ChunkStore& out) {
  const int64_t nrows = (int64_t)rp.size() - 1;
  const int nchunk = (int)std::max<int64_t>(1, (ncols + cw - 1) / cw);
  std::vector<int64_t> cnt((size_t)nchunk * nrows, 0);
  for (int64_t r = 0; r < nrows; ++r)
    for (int64_t q = rp[r]; q < rp[r + 1]; ++q) cnt[(size_t)(col[q] / cw) * nrows + r]++;
  std::vector<int32_t>& crp = out.rowptr;
  crp.assign((size_t)nchunk * (nrows + 1), 0);
  out.nnz.assign(nchunk, 0);
  int64_t off = 0;
  for (int c = 0; c < nchunk; ++c) {
    for (int64_t r = 0; r < nrows; ++r) {
      crp[(size_t)c * (nrows + 1) + r] = (int32_t)off;
      off += (cnt[(size_t)c * nrows + r] + 1) & ~int64_t(1);
      if (off * 8 >= (int64_t(1) << 31)) {   // byte offsets of the kernels' buffer loads
        h->err = "blocked operator exceeds 2^28 stored entries";
        return QP_ERR_UNSUPPORTED;
      }
    }
    crp[(size_t)c * (nrows + 1) + nrows] = (int32_t)off;
    out.nnz[c] = crp[(size_t)c * (nrows + 1) + nrows] - crp[(size_t)c * (nrows + 1)];
  }
  out.nchunk = nchunk;
  out.stored = off;
  out.col.assign(off, 0);
  out.val.assign(off, 0.0);
  std::vector<int64_t> cur(cnt.size());
  for (int c = 0; c < nchunk; ++c)
    for (int64_t r = 0; r < nrows; ++r) cur[(size_t)c * nrows + r] = crp[(size_t)c * (nrows + 1) + r];
  for (int64_t r = 0; r < nrows; ++r)
    for (int64_t q = rp[r]; q < rp[r + 1]; ++q) {
      const int c = col[q] / cw;
      const int64_t pos = cur[(size_t)c * nrows + r]++;
      out.col[pos] = (uint16_t)(col[q] - c * cw);
      out.val[pos] = val[q];
    }
  return QP_OK;
}

static qp_status build_chunked(qp_handle h, qp_handle_s::Chunked& ck, const std::vector<int32_t>& rp,
                               const std::vector<int32_t>& col, const std::vector<double>& val,
                               int ncols, int cw_default, int kv_default, bool row_side,
                               const char* env, const char* env_lpr, const char* env_kv) {
  const int64_t rows_in = (int64_t)rp.size() - 1;
  // Chunk width (columns staged in LDS per block); `env` overrides it.  A
  // work item holds at least one (chunk, row) segment, so few long rows (a
  // handful of dense rows over many columns) get narrower chunks until there
  // are segments for two blocks per CU.
  int cw = cw_default;
  while (cw > 1024 && rows_in * ((ncols + cw - 1) / cw) < 512) cw = std::max(1024, cw / 2) & ~1;
  if (const char* e = std::getenv(env)) {
    const int v = std::atoi(e);
    if (v >= 1024 && v <= kChunkCols) cw = v & ~1;
  }
  const int per_cu = std::max(1, (int)(163840 / (8 * (int64_t)cw + 1024)));
  const int64_t nrows = (int64_t)rp.size() - 1;
  const int64_t nnz = rp[nrows];
  ChunkStore cs;
  CHK(chunk_store(h, rp, col, val, ncols, cw, cs));
  const int nchunk = cs.nchunk;
  const int64_t stored = cs.stored;
  const std::vector<int32_t>& crp = cs.rowptr;
  const std::vector<int64_t>& cnnz = cs.nnz;
  // work items: per chunk, proportional to its entries, rows cut at equal entry counts.
  // A pass writes one partial slot per work item and the PCG kernels sum at
  // most kGridMax of them: chunk i gets at most 1 + target * (its share of the
  // entries) items, so target <= kGridMax - nchunk keeps the count in range.
  if (nchunk > kGridMax / 2) {
    h->err = "blocked operator: too many column chunks (" + std::to_string(nchunk) + ")";
    return QP_ERR_UNSUPPORTED;
  }
  const int target = std::min(kGridMax - nchunk, std::max(nchunk, 256 * per_cu - nchunk));
  std::vector<int32_t> work;
  for (int c = 0; c < nchunk; ++c) {
    const int items =
        (int)std::max<int64_t>(1, stored > 0 ? (int64_t)target * cnnz[c] / stored : 1);
    const int32_t* base = &crp[(size_t)c * (nrows + 1)];
    int64_t r = 0;
    for (int it = 0; it < items; ++it) {
      const int64_t goal = base[0] + (cnnz[c] * (it + 1)) / items;
      int64_t r1 = r;
      while (r1 < nrows && (base[r1 + 1] <= goal || r1 == r)) ++r1;
      if (it == items - 1) r1 = nrows;
      if (r1 > r || it == items - 1) {
        work.push_back(c);
        work.push_back((int32_t)r);
        work.push_back((int32_t)r1);
      }
      r = r1;
      if (r >= nrows) break;
    }
  }
  if ((int64_t)(work.size() / 3) > kGridMax) {
    h->err = "blocked operator: more work items than partial-sum slots";
    return QP_ERR_UNSUPPORTED;
  }
  ck.nrows = (int)nrows;
  ck.ncols = ncols;
  ck.nchunk = nchunk;
  ck.chunk_cols = cw;
  ck.nwork = (int)(work.size() / 3);
  ck.nnz = nnz;
  ck.stored = stored;
  const double avg = nrows > 0 ? (double)nnz / ((double)nrows * nchunk) : 1.0;
  // multi-chunk passes stage straight into LDS: 64 VGPRs, two blocks per CU
  ck.kv = nchunk > 1 ? 1 : kv_default;
  if (const char* e = std::getenv(env_kv)) ck.kv = std::atoi(e) & 1;
  // Lanes per row.  A float64 pass staged through registers (kv 0) takes eight
  // entry pairs per lane at up to 8 lanes per row, the others four (see
  // k_chunked): size the group so one batch covers a typical row, the
  // single-chunk row side (the hot one, float64) generously, else about four
  // entries per lane.  On that row side 4 lanes of 16 entries, then 16 or
  // more lanes of 8: for rows of about 100 entries, 16 lanes of 8 measured
  // 39.9 us against 41.3 us for 8 lanes of 16.
  ck.lpr = pow2_clamp(avg / 4.0, 4, 64);
  if (row_side && nchunk == 1 && h->vk == VK_F64 && ck.kv == 0) {
    ck.lpr = 4;
    while (ck.lpr < 64 && ck.lpr * (ck.lpr <= 4 ? 16 : 8) < avg) ck.lpr *= 2;
  }
  if (const char* e = std::getenv(env_lpr)) ck.lpr = pow2_clamp(std::atof(e), 4, 64);
  if (const char* e = std::getenv("QPK_XCD_MAP")) ck.xcd_map = std::atoi(e) != 0;
  CHK(upload(h, &ck.work, work.data(), (int64_t)work.size()));
  CHK(upload(h, &ck.rowptr, crp.data(), (int64_t)crp.size()));
  CHK(upload(h, &ck.col, cs.col.data(), stored));
  CHK(upload(h, &ck.val, cs.val.data(), stored));
  if (h->vk != VK_F64) CHK(upload_lo(h, &ck.val_lo, cs.val));
  if (nchunk > 1) CHK(dalloc_t(h, &ck.partial, (int64_t)nchunk * nrows));
  HIPCHK(hipStreamSynchronize(h->st));  // host staging vectors go out of scope
  ck.on = true;
  return QP_OK;
}

// The fused single-read product's layout: the rows of the blocked row side
// (rows of P, then those of A unless they are folded into P's twins) with
// their columns cut in two halves of at most kFusedHalfMax, and row ranges of
// equal entry counts, one per pair of blocks (one block per CU).  Used for
// H = P^T W P when n <= 2 kFusedHalfMax and the operator is large enough for
// the pass to stream (QPK_FUSED=0 never, =1 whenever the shape allows).
static qp_status build_fused(qp_handle h, const std::vector<int32_t>& rp, const std::vector<int32_t>& col,
                             const std::vector<double>& val, int ncols, const std::vector<int32_t>& twin,
                             const double* lA, const double* uA) {
  const int64_t nrows = (int64_t)rp.size() - 1;
  const char* e = std::getenv("QPK_FUSED");
  const int mode = e ? std::atoi(e) : -1;
  if (mode == 0 || h->h_kind != QP_H_PTWP || ncols > 2 * kFusedHalfMax || nrows < 1) return QP_OK;
  if (mode < 0 && rp[nrows] < (int64_t(1) << 22)) return QP_OK;
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int nrange = (int)std::max<int64_t>(1, std::min<int64_t>(cus / 2, nrows));
  if (2 * nrange > kGridMax) return QP_OK;
  const int half = (((ncols + 1) / 2) + 1) & ~1;   // even, >= ncols - half
  ChunkStore cs;
  CHK(chunk_store(h, rp, col, val, ncols, half, cs));
  if (cs.nchunk > 2) return QP_OK;
  if (cs.nchunk == 1) {   // ncols <= half: an empty second half
    cs.rowptr.resize(2 * (size_t)(nrows + 1), (int32_t)cs.stored);
    cs.nnz.push_back(0);
  }
  // row ranges of equal stored entries over both halves
  std::vector<int32_t> range(nrange + 1, (int32_t)nrows);
  range[0] = 0;
  {
    const int32_t* r0 = cs.rowptr.data();
    const int32_t* r1 = cs.rowptr.data() + (nrows + 1);
    const int64_t total = cs.stored;
    int64_t acc = 0;
    int next = 1;
    for (int64_t r = 0; r < nrows && next < nrange; ++r) {
      acc += (r0[r + 1] - r0[r]) + (r1[r + 1] - r1[r]);
      while (next < nrange && acc * nrange >= total * next) range[next++] = (int32_t)(r + 1);
    }
  }
  qp_handle_s::Fused& fz = h->fz;
  fz.nrows = (int)nrows;
  fz.half = half;
  fz.nrange = nrange;
  fz.stored = cs.stored;
  // per row the row of A it carries (its twin, or itself after the rows of
  // P), with the finite sides of that row as flag bits
  std::vector<int32_t> info((size_t)nrows, -1);
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = r < h->p_rows ? (twin.empty() ? -1 : twin[r]) : r - h->p_rows;
    if (i < 0) continue;
    if (i >= (1 << 29)) {
      h->err = "fused layout: too many rows of A";
      return QP_ERR_UNSUPPORTED;
    }
    info[r] = (int32_t)i | (std::isfinite(lA[i]) ? (1 << 30) : 0) | (std::isfinite(uA[i]) ? (1 << 29) : 0);
  }
  CHK(upload(h, &fz.rowinfo, info.data(), nrows));
  CHK(upload(h, &fz.range, range.data(), (int64_t)range.size()));
  CHK(upload(h, &fz.rowptr, cs.rowptr.data(), (int64_t)cs.rowptr.size()));
  CHK(upload(h, &fz.col, cs.col.data(), cs.stored));
  CHK(upload(h, &fz.val, cs.val.data(), cs.stored));
  if (h->vk != VK_F64) CHK(upload_lo(h, &fz.val_lo, cs.val));
  CHK(dalloc_t(h, &fz.xch, 4 * nrows));
  // every exchange slot starts empty (all bits set)
  HIPCHK(hipMemsetAsync(fz.xch, 0xff, sizeof(double) * 4 * nrows, h->st));
  CHK(dalloc_t(h, &fz.ypart, (int64_t)nrange * ncols));
  if (const char* sm = std::getenv("QPK_FUSED_SPIN")) fz.spin_max = std::max(1, std::atoi(sm));
  HIPCHK(fused_set_attributes());
  HIPCHK(hipStreamSynchronize(h->st));  // host staging vectors go out of scope
  fz.on = true;
  return QP_OK;
}

static qp_status create_impl(qp_handle h, const qp_desc* d) {
  const int64_t n = d->n, m = d->m, me = d->me;
  auto bad = [&](const std::string& msg) { h->err = msg; return QP_ERR_ARG; };
  if (n <= 0 || m < 0 || me < 0 || me > 64) return bad("need n >= 1, m >= 0, 0 <= me <= 64");
  if (d->precision < QP_PREC_FP64 || d->precision > QP_PREC_BF16_ACC64) return bad("bad precision");
  if (!d->c) return bad("c is required");
  if (me > 0 && (!d->C || !d->b)) return bad("C and b are required when me > 0");
  if (m > 0 && (!d->lA || !d->uA)) return bad("lA and uA are required when m > 0");
  if (m > 0 && d->a_kind != QP_A_DENSE && d->a_kind != QP_A_CSR) return bad("m > 0 needs A");
  if (m == 0 && d->a_kind != QP_A_NONE && d->a_kind != QP_A_DENSE && d->a_kind != QP_A_CSR)
    return bad("bad a_kind");
  h->n = (int)n; h->m = (int)m; h->me = (int)me; h->h_kind = d->h_kind; h->prec = d->precision;
  switch (d->precision) {
    case QP_PREC_FP32: h->vk = VK_F32; break;
    case QP_PREC_BF16: h->vk = VK_BF16; break;
    case QP_PREC_FP32_ACC64: h->vk = VK_F32X; break;
    case QP_PREC_BF16_ACC64: h->vk = VK_BF16X; break;
    default: h->vk = VK_F64; break;
  }
  auto finite_all = [](const double* p, int64_t cnt) {
    for (int64_t i = 0; i < cnt; ++i) if (!std::isfinite(p[i])) return false;
    return true;
  };
  if (!finite_all(d->c, n)) return bad("c has non-finite entries");
  // bounds
  std::vector<double> lx(n, -INFINITY), ux(n, INFINITY);
  if (d->lx) std::copy(d->lx, d->lx + n, lx.begin());
  if (d->ux) std::copy(d->ux, d->ux + n, ux.begin());
  for (int64_t j = 0; j < n; ++j) {
    if (std::isnan(lx[j]) || std::isnan(ux[j]) || lx[j] == INFINITY || ux[j] == -INFINITY)
      return bad("invalid variable bound at " + std::to_string(j));
    if (std::isfinite(lx[j]) && std::isfinite(ux[j]) && !(lx[j] < ux[j]))
      return bad("need lx < ux where both are finite (variable " + std::to_string(j) + ")");
  }
  for (int64_t i = 0; i < m; ++i) {
    const double l = d->lA[i], u = d->uA[i];
    if (std::isnan(l) || std::isnan(u) || l == INFINITY || u == -INFINITY || l > u)
      return bad("invalid row bounds at row " + std::to_string(i));
  }
  if (me > 0 && (!finite_all(d->C, me * n) || !finite_all(d->b, me))) return bad("C or b non-finite");

  // Hessian pieces
  std::vector<double> diagH(n, 0.0), h0(n, 0.0);
  int64_t k = 0;
  int64_t p_rows = 0;
  std::vector<int64_t> prp;
  const int32_t* pcol = nullptr;
  const double* pval = nullptr;
  if (d->h_kind == QP_H_DENSE) {
    if (!d->H || !finite_all(d->H, n * n)) return bad("dense H missing or non-finite");
    for (int64_t j = 0; j < n; ++j) diagH[j] = d->H[j * n + j];
  } else if (d->h_kind == QP_H_LOWRANK) {
    k = d->k;
    if (k < 1 || k > 1024 || !d->U || !d->wd || !d->h0) return bad("low-rank H needs 1 <= k <= 1024, h0, U, wd");
    if (!finite_all(d->U, n * k) || !finite_all(d->wd, k) || !finite_all(d->h0, n))
      return bad("low-rank H has non-finite entries");
    for (int64_t j = 0; j < n; ++j) h0[j] = d->h0[j];
    diagH = h0;
  } else if (d->h_kind == QP_H_PTWP) {
    p_rows = d->p_rows;
    if (p_rows < 1 || !d->p_rowptr || !d->p_col || !d->p_val || !d->p_w) return bad("P^T W P needs P and w");
    if (d->p_rowptr[0] != 0) return bad("P rowptr[0] must be 0");
    for (int64_t v = 0; v < p_rows; ++v)
      if (d->p_rowptr[v + 1] < d->p_rowptr[v]) return bad("P rowptr not monotone");
    const int64_t nnz = d->p_rowptr[p_rows];
    for (int64_t q = 0; q < nnz; ++q)
      if (d->p_col[q] < 0 || d->p_col[q] >= n || !std::isfinite(d->p_val[q])) return bad("bad P entry");
    for (int64_t v = 0; v < p_rows; ++v)
      if (!(d->p_w[v] > 0.0) || !std::isfinite(d->p_w[v]) || (d->p_d && !std::isfinite(d->p_d[v])))
        return bad("P weights must be positive and finite");
    prp.assign(d->p_rowptr, d->p_rowptr + p_rows + 1);
    pcol = d->p_col;
    pval = d->p_val;
  } else {
    return bad("bad h_kind");
  }
  h->k = (int)k;
  h->p_rows = (int)p_rows;
  h->nRP = (int)(p_rows + m);

  // A as CSR rows (dense A keeps its nonzeros)
  std::vector<int64_t> arp(m + 1, 0);
  std::vector<int32_t> acol;
  std::vector<double> aval;
  if (m > 0) {
    if (d->a_kind == QP_A_DENSE) {
      if (!d->A || !finite_all(d->A, m * n)) return bad("dense A missing or non-finite");
      for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
          const double v = d->A[i * n + j];
          if (v != 0.0) { acol.push_back((int32_t)j); aval.push_back(v); }
        }
        arp[i + 1] = (int64_t)acol.size();
      }
    } else {
      if (!d->a_rowptr || !d->a_col || !d->a_val || d->a_rowptr[0] != 0) return bad("bad CSR A");
      for (int64_t i = 0; i < m; ++i) {
        if (d->a_rowptr[i + 1] < d->a_rowptr[i]) return bad("A rowptr not monotone");
        for (int64_t q = d->a_rowptr[i]; q < d->a_rowptr[i + 1]; ++q) {
          if (d->a_col[q] < 0 || d->a_col[q] >= n || !std::isfinite(d->a_val[q])) return bad("bad A entry");
          acol.push_back(d->a_col[q]);
          aval.push_back(d->a_val[q]);
        }
        arp[i + 1] = (int64_t)acol.size();
      }
    }
  }
  const int64_t pnnz = p_rows > 0 ? prp[p_rows] : 0;
  const int64_t annz = (int64_t)acol.size();
  const int64_t hnnz = d->h_kind == QP_H_DENSE ? n * n : 0;
  if (pnnz + annz >= INT32_MAX || pnnz + annz + hnnz >= INT32_MAX)
    return bad("operators exceed 2^31 stored entries");
  h->nnz_rp = pnnz + annz;

  // Row side RP = [P rows; A rows]
  std::vector<int32_t> rrp(h->nRP + 1), rcol(h->nnz_rp);
  std::vector<double> rval(h->nnz_rp);
  for (int64_t v = 0; v < p_rows; ++v) {
    rrp[v] = (int32_t)prp[v];
    for (int64_t q = prp[v]; q < prp[v + 1]; ++q) { rcol[q] = pcol[q]; rval[q] = pval[q]; }
  }
  for (int64_t i = 0; i <= m; ++i) rrp[p_rows + i] = (int32_t)(pnnz + arp[i]);
  for (int64_t q = 0; q < annz; ++q) { rcol[pnnz + q] = acol[q]; rval[pnnz + q] = aval[q]; }

  // Column side XS: per variable j, [H row j | column j of P | column j of A]
  std::vector<int64_t> cnt_h(n, 0), cnt_p(n, 0), cnt_a(n, 0);
  if (hnnz) for (int64_t j = 0; j < n; ++j) cnt_h[j] = n;
  for (int64_t q = 0; q < pnnz; ++q) cnt_p[pcol[q]]++;
  for (int64_t q = 0; q < annz; ++q) cnt_a[acol[q]]++;
  std::vector<int32_t> xrp(n + 1), xs1(n), xs2(n);
  int64_t acc = 0;
  for (int64_t j = 0; j < n; ++j) {
    xrp[j] = (int32_t)acc; acc += cnt_h[j];
    xs1[j] = (int32_t)acc; acc += cnt_p[j];
    xs2[j] = (int32_t)acc; acc += cnt_a[j];
  }
  xrp[n] = (int32_t)acc;
  h->nnz_xs = acc;
  std::vector<int32_t> xcol(acc);
  std::vector<double> xval(acc);
  {
    std::vector<int64_t> fp(n), fa(n);
    for (int64_t j = 0; j < n; ++j) {
      if (hnnz) for (int64_t i = 0; i < n; ++i) { xcol[xrp[j] + i] = (int32_t)i; xval[xrp[j] + i] = d->H[j * n + i]; }
      fp[j] = xs1[j];
      fa[j] = xs2[j];
    }
    for (int64_t v = 0; v < p_rows; ++v)
      for (int64_t q = prp[v]; q < prp[v + 1]; ++q) {
        const int64_t j = pcol[q];
        xcol[fp[j]] = (int32_t)v; xval[fp[j]] = pval[q]; fp[j]++;
      }
    for (int64_t i = 0; i < m; ++i)
      for (int64_t q = arp[i]; q < arp[i + 1]; ++q) {
        const int64_t j = acol[q];
        xcol[fa[j]] = (int32_t)i; xval[fa[j]] = aval[q]; fa[j]++;
      }
  }
  h->has_xs = acc > 0;
  h->has_ts = k > 0 || me > 0;

  // LDS-staged blocked copies of the two PCG matvec operators.  The column
  // side needs one gathered vector per entry, so it is built when H has no
  // dense or low-rank part: its columns index [u (p_rows) | wA (m)].
  const bool want_ck_x = acc > 0 && hnnz == 0 && k == 0;
  std::vector<int32_t> scol;
  if (want_ck_x) {
    scol.resize(acc);
    for (int64_t j = 0; j < n; ++j) {
      for (int64_t q = xs1[j]; q < xs2[j]; ++q) scol[q] = xcol[q];
      for (int64_t q = xs2[j]; q < xrp[j + 1]; ++q) scol[q] = (int32_t)(p_rows + xcol[q]);
    }
  }

  // Rows of A that repeat rows of P (the radiation-therapy form: the max-dose
  // rows are rows of the dose matrix).  When every row of A has its own twin,
  // the blocked passes hold P alone (QPK_FOLD_A=0 keeps A in them).
  std::vector<int32_t> twin;
  if (want_ck_x && p_rows > 0 && m > 0) {
    const char* e = std::getenv("QPK_FOLD_A");
    if (!(e && std::atoi(e) == 0))
      h->fold_a = match_twins(p_rows, prp, pcol, pval, m, arp, acol, aval, twin);
  }

  // Launch shapes
  const double avg_r = h->nRP > 0 ? (double)h->nnz_rp / h->nRP : 0.0;
  const double avg_x = (double)acc / n + (double)k;
  h->lpr_r = pow2_clamp(avg_r / 4.0, 4, 64);
  h->lpr_x = pow2_clamp(avg_x / 4.0, 4, 64);
  h->g_r = grid_cap((int64_t)h->nRP * h->lpr_r, kBlock, kGridMax);
  h->g_ra = grid_cap((int64_t)std::max<int64_t>(m, 1) * h->lpr_r, kBlock, kGridMax);
  h->g_x = grid_cap(n * (int64_t)h->lpr_x, kBlock, kGridMax);
  h->g_vec = grid_cap(h->N(), kBlock, 512);
  h->g_rmv = h->g_r;
  h->g_xmv = h->g_x;
  h->g_n = grid_cap(n, kBlock, kGridMax);
  h->g_ts = (int)std::max<int64_t>(1, std::min<int64_t>(kGridMax, (n + 63) / 64));
  h->ts_chunk = (int)((n + h->g_ts - 1) / h->g_ts);

  // Device buffers
  CHK(upload(h, &h->rp_rowptr, rrp.data(), (int64_t)rrp.size()));
  CHK(upload(h, &h->rp_col, rcol.data(), (int64_t)rcol.size()));
  CHK(upload(h, &h->rp_val, rval.data(), (int64_t)rval.size()));
  CHK(upload(h, &h->xs_rowptr, xrp.data(), (int64_t)xrp.size()));
  CHK(upload(h, &h->xs_seg1, xs1.data(), (int64_t)xs1.size()));
  CHK(upload(h, &h->xs_seg2, xs2.data(), (int64_t)xs2.size()));
  CHK(upload(h, &h->xs_col, xcol.data(), (int64_t)xcol.size()));
  CHK(upload(h, &h->xs_val, xval.data(), (int64_t)xval.size()));
  HIPCHK(chunked_set_attributes());
  // Row side: one chunk covering every column when it fits the LDS (the row
  // epilogue then runs in place), staged through registers.  Column side:
  // half-LDS chunks staged straight into LDS, two blocks per CU (both
  // measured fastest on the radiation-therapy workload).
  if (h->fold_a) {
    // row side: the P rows of RP; column side: XS without its A segments
    const std::vector<int32_t> rrp_p(rrp.begin(), rrp.begin() + p_rows + 1);
    std::vector<int32_t> xrp_p(n + 1), scol_p;
    std::vector<double> xval_p;
    scol_p.reserve((size_t)pnnz);
    xval_p.reserve((size_t)pnnz);
    for (int64_t j = 0; j < n; ++j) {
      xrp_p[j] = (int32_t)scol_p.size();
      for (int64_t q = xs1[j]; q < xs2[j]; ++q) {
        scol_p.push_back(scol[q]);
        xval_p.push_back(xval[q]);
      }
    }
    xrp_p[n] = (int32_t)scol_p.size();
    CHK(build_chunked(h, h->ck_r, rrp_p, rcol, rval, (int)n, kChunkCols, 0, true, "QPK_CHUNK_COLS_R",
                      "QPK_LPR_R", "QPK_KV_R"));
    CHK(build_chunked(h, h->ck_x, xrp_p, scol_p, xval_p, (int)p_rows, kChunkCols / 2, 1, false,
                      "QPK_CHUNK_COLS_X", "QPK_LPR_X", "QPK_KV_X"));
    CHK(upload(h, &h->twin, twin.data(), (int64_t)twin.size()));
    CHK(build_fused(h, rrp_p, rcol, rval, (int)n, twin, d->lA, d->uA));
  } else {
    if (h->nRP > 0)
      CHK(build_chunked(h, h->ck_r, rrp, rcol, rval, (int)n, kChunkCols, 0, true, "QPK_CHUNK_COLS_R",
                        "QPK_LPR_R", "QPK_KV_R"));
    if (h->nRP > 0 && want_ck_x) CHK(build_fused(h, rrp, rcol, rval, (int)n, {}, d->lA, d->uA));
    if (want_ck_x)
      CHK(build_chunked(h, h->ck_x, xrp, scol, xval, (int)(p_rows + m), kChunkCols / 2, 1, false,
                        "QPK_CHUNK_COLS_X", "QPK_LPR_X", "QPK_KV_X"));
  }
  if (const char* e = std::getenv("QPK_ALTERNATE")) h->alternate = std::atoi(e) != 0;
  h->g_epi_r = grid_cap(std::max<int64_t>(h->nRP, 1), kBlock, kGridMax);
  h->g_epi_x = grid_cap(n, kBlock, kGridMax);
  if (h->ck_r.on) h->g_rmv = h->ck_r.nchunk == 1 ? h->ck_r.nwork : h->g_epi_r;
  if (h->ck_x.on) h->g_xmv = h->ck_x.nchunk == 1 ? h->ck_x.nwork : h->g_epi_x;
  if (h->fz.on || pcg_fuses_epilogue(h)) {
    // the PCG update then sums the x-part of q from partials, 16 entries per
    // wave: one wave per task (k_cg_update_split)
    const int64_t tasks = (n + 15) / 16 + (h->N() - n + 63) / 64;
    h->g_vec = (int)std::min<int64_t>(kGridMax, std::max<int64_t>(h->g_vec, (tasks + 3) / 4));
  }
  if (k > 0) {
    CHK(upload(h, &h->U, d->U, n * k));
    CHK(upload(h, &h->wd, d->wd, k));
  } else {
    CHK(dalloc_t(h, &h->U, 1));
    CHK(dalloc_t(h, &h->wd, 1));
  }
  if (h->vk != VK_F64) {
    CHK(upload_lo(h, &h->rp_lo, rval));
    CHK(upload_lo(h, &h->xs_lo, xval));
    if (k > 0) {
      std::vector<double> uv(d->U, d->U + n * k);
      CHK(upload_lo(h, &h->U_lo, uv));
    } else {
      h->U_lo = h->U;
    }
  }
  CHK(upload(h, &h->h0, h0.data(), n));
  CHK(upload(h, &h->c, d->c, n));
  CHK(dalloc_t(h, &h->c_eff, n));
  CHK(upload(h, &h->lx, lx.data(), n));
  CHK(upload(h, &h->ux, ux.data(), n));
  if (m > 0) {
    CHK(upload(h, &h->lA, d->lA, m));
    CHK(upload(h, &h->uA, d->uA, m));
  } else {
    CHK(dalloc_t(h, &h->lA, 1));
    CHK(dalloc_t(h, &h->uA, 1));
  }
  if (me > 0) {
    CHK(upload(h, &h->Cm, d->C, me * n));
    CHK(upload(h, &h->b, d->b, me));
  } else {
    CHK(dalloc_t(h, &h->Cm, 1));
    CHK(dalloc_t(h, &h->b, 1));
  }
  if (p_rows > 0) {
    CHK(upload(h, &h->pw, d->p_w, p_rows));
    if (d->p_d) CHK(upload(h, &h->pd, d->p_d, p_rows));
  } else {
    CHK(dalloc_t(h, &h->pw, 1));
  }
  CHK(dalloc_t(h, &h->diagH, n));

  const int64_t N = h->N();
  CHK(dalloc_t(h, &h->x, n));
  CHK(dalloc_t(h, &h->lam, h->nlam()));
  CHK(dalloc_t(h, &h->s, h->ns()));
  CHK(dalloc_t(h, &h->res, h->nres()));
  CHK(dalloc_t(h, &h->rhs, N));
  CHK(dalloc_t(h, &h->jdiag, N));
  CHK(dalloc_t(h, &h->dl, me + 2 * m));
  CHK(dalloc_t(h, &h->qdiag, n));
  CHK(dalloc_t(h, &h->uw, p_rows + m));
  h->wA_mv = h->uw + p_rows;
  CHK(dalloc_t(h, &h->wA_res, m));
  CHK(dalloc_t(h, &h->wA_rhs, m));
  CHK(dalloc_t(h, &h->jw, m));
  CHK(dalloc_t(h, &h->we_mv, me));
  CHK(dalloc_t(h, &h->we_res, me));
  CHK(dalloc_t(h, &h->we_rhs, me));
  CHK(dalloc_t(h, &h->te, me));
  CHK(dalloc_t(h, &h->g, k));
  h->u = h->uw;
  CHK(dalloc_t(h, &h->cg_r, N));
  CHK(dalloc_t(h, &h->cg_z, N));
  CHK(dalloc_t(h, &h->cg_p, N));
  if (const char* e = std::getenv("QPK_GRAPH")) h->gr.enabled = std::atoi(e) != 0;
  CHK(dalloc_t(h, &h->cg_q, N));
  CHK(dalloc_t(h, &h->tmp, N));
  CHK(dalloc_t(h, &h->arhs, N));
  CHK(dalloc_t(h, &h->valign, N));
  CHK(dalloc_t(h, &h->dir, n + h->nlam()));
  CHK(dalloc_t(h, &h->ds_w, h->ns()));
  CHK(dalloc_t(h, &h->part, (int64_t)P_COUNT * kGridMax));
  CHK(dalloc_t(h, &h->ts_part, (int64_t)h->g_ts * (k + me)));
  CHK(dalloc_t(h, &h->sc, S_COUNT));
  CHK(dalloc_t(h, &h->fl, F_COUNT));
  HIPCHK(hipMemsetAsync(h->part, 0, sizeof(double) * P_COUNT * kGridMax, h->st));
  HIPCHK(hipMemsetAsync(h->dir, 0, sizeof(double) * (n + h->nlam()), h->st));
  HIPCHK(hipMemsetAsync(h->ds_w, 0, sizeof(double) * h->ns(), h->st));
  HIPCHK(hipMemsetAsync(h->fl, 0, sizeof(int) * F_COUNT, h->st));
  HIPCHK(hipMemsetAsync(h->sc, 0, sizeof(double) * S_COUNT, h->st));
  {
    hipError_t e1 = hipHostMalloc((void**)&h->hsc, sizeof(double) * S_COUNT, hipHostMallocDefault);
    hipError_t e2 = hipHostMalloc((void**)&h->hfl, sizeof(int) * F_COUNT, hipHostMallocDefault);
    hipError_t e3 = hipHostMalloc((void**)&h->hpoll, 2 * sizeof(int) * F_COUNT, hipHostMallocDefault);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      h->err = "hipHostMalloc failed";
      return QP_ERR_ALLOC;
    }
    for (hipEvent_t& e : h->poll_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }

  CHK(upload(h, &h->diagH0, diagH.data(), n));
  CHK(derive_constants(h));
  CHK(run_init_state(h, 1.0));
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_create(const qp_desc* d, void* stream, qp_handle* out) {
  if (!out) return QP_ERR_ARG;
  *out = nullptr;
  if (!d) return QP_ERR_ARG;
  qp_handle h = new (std::nothrow) qp_handle_s();
  if (!h) return QP_ERR_ALLOC;
  h->st = (hipStream_t)stream;
  qp_status s;
  try {
    s = create_impl(h, d);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    s = QP_ERR_ALLOC;
  } catch (...) {
    h->err = "unexpected host exception";
    s = QP_ERR_ARG;
  }
  if (s != QP_OK) {
    // the handle is gone: keep the message for qp_last_error(NULL)
    g_create_error = h->err;
    delete h;
    return s;
  }
  *out = h;
  return QP_OK;
}

void qp_destroy(qp_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->st);
  delete h;
}

qp_status qp_set_stream(qp_handle h, void* stream) {
  if (!h) return QP_ERR_ARG;
  h->st = (hipStream_t)stream;
  return QP_OK;
}

qp_status qp_sizes(qp_handle h, int64_t* n_x, int64_t* n_lam, int64_t* n_s, int64_t* n_kkt,
                   int64_t* n_res) {
  if (!h) return QP_ERR_ARG;
  if (n_x) *n_x = h->n;
  if (n_lam) *n_lam = h->nlam();
  if (n_s) *n_s = h->ns();
  if (n_kkt) *n_kkt = h->N();
  if (n_res) *n_res = h->nres();
  return QP_OK;
}

qp_status qp_set_state(qp_handle h, const double* x, const double* lam, const double* s, double mu) {
  if (!h) return QP_ERR_ARG;
  if (!x || !lam || !s) { h->err = "x, lam and s are required"; return QP_ERR_ARG; }
  if (!(mu > 0.0) || !std::isfinite(mu)) { h->err = "mu must be positive"; return QP_ERR_ARG; }
  HIPCHK(hipMemcpyAsync(h->x, x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipMemcpyAsync(h->lam, lam, sizeof(double) * h->nlam(), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipMemcpyAsync(h->s, s, sizeof(double) * h->ns(), hipMemcpyDeviceToDevice, h->st));
  h->mu = mu;
  h->res_valid = h->sys_valid = false;
  h->solved = false;
  VecArgs v = vec_args(h);
  const int grid = grid_cap(h->nlam(), kBlock, kGridMax);
  HIPCHK(launch_check_state(v, grid, h->st));
  HIPCHK(launch_finish_sum(h->part + P_CHK * kGridMax, grid, h->sc + S_RELRES, h->st));
  CHK(read_back(h));
  if (h->hsc[S_RELRES] != 0.0) {
    h->err = "state has non-positive or non-finite slacks/multipliers (" +
             std::to_string((long long)h->hsc[S_RELRES]) + " entries)";
    return QP_ERR_ARG;
  }
  return QP_OK;
}

qp_status qp_get_state(qp_handle h, double* x, double* lam, double* s, double* mu) {
  if (!h) return QP_ERR_ARG;
  if (x) HIPCHK(hipMemcpyAsync(x, h->x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->st));
  if (lam) HIPCHK(hipMemcpyAsync(lam, h->lam, sizeof(double) * h->nlam(), hipMemcpyDeviceToDevice, h->st));
  if (s) HIPCHK(hipMemcpyAsync(s, h->s, sizeof(double) * h->ns(), hipMemcpyDeviceToDevice, h->st));
  if (mu) *mu = h->mu;
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_init_state(qp_handle h, double mu) {
  if (!h) return QP_ERR_ARG;
  if (!(mu > 0.0)) { h->err = "mu must be positive"; return QP_ERR_ARG; }
  CHK(run_init_state(h, mu));
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_residuals(qp_handle h, double* r, double* norms) {
  if (!h) return QP_ERR_ARG;
  CHK(run_residuals(h));
  if (r) HIPCHK(hipMemcpyAsync(r, h->res, sizeof(double) * h->nres(), hipMemcpyDeviceToDevice, h->st));
  CHK(read_back(h));
  if (norms) {
    norms[0] = h->hsc[S_NORM];
    norms[1] = h->hsc[S_PRIMAL];
    norms[2] = h->hsc[S_DUAL];
    norms[3] = h->hsc[S_COMPL];
  }
  return QP_OK;
}

qp_status qp_newton_rhs(qp_handle h, double* rhs, double* jacobi_diag) {
  if (!h) return QP_ERR_ARG;
  CHK(prepare(h));
  if (rhs) HIPCHK(hipMemcpyAsync(rhs, h->rhs, sizeof(double) * h->N(), hipMemcpyDeviceToDevice, h->st));
  if (jacobi_diag)
    HIPCHK(hipMemcpyAsync(jacobi_diag, h->jdiag, sizeof(double) * h->N(), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_kkt_matvec(qp_handle h, const double* v, double* y) {
  if (!h || !v || !y) return QP_ERR_ARG;
  CHK(prepare(h));
  const bool fused = fused_active(h);
  CHK(run_matvec(h, false, v, y, nullptr, nullptr));
  if (fused) {
    CHK(read_back(h));
    if (h->hfl[F_FUSEFAIL]) {   // a block pair timed out: redo it with the two-pass kernels
      h->fz.failed = true;
      CHK(run_matvec(h, false, v, y, nullptr, nullptr));
    }
  }
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

static pcg_options pcg_opts_or_default(const pcg_options* o) {
  pcg_options d;
  qp_default_pcg_options(&d);
  if (!o) return d;
  d = *o;
  if (!(d.tol > 0.0)) d.tol = 1e-7;
  if (d.maxit < 1) d.maxit = 5000;
  if (d.check_every < 1) d.check_every = 8;
  return d;
}

qp_status kkt_pcg_solve(qp_handle h, const double* rhs, double* sol, const pcg_options* o,
                        pcg_info* info) {
  if (!h || !rhs || !sol) return QP_ERR_ARG;
  CHK(prepare(h));
  const pcg_options po = pcg_opts_or_default(o);
  pcg_info inf{};
  qp_status s = run_pcg(h, rhs, sol, po, &inf);
  if (info) *info = inf;
  return s;
}

qp_status qp_newton_direction(qp_handle h, const pcg_options* o, double* dx, double* dlam,
                              double* ds, pcg_info* info) {
  if (!h) return QP_ERR_ARG;
  CHK(prepare(h));
  const pcg_options po = pcg_opts_or_default(o);
  pcg_info inf{};
  qp_status s = run_pcg(h, h->rhs, h->dir, po, &inf);
  if (info) *info = inf;
  if (s != QP_OK) return s;
  CHK(run_recover(h, 0.99));
  if (dx) HIPCHK(hipMemcpyAsync(dx, h->dir, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->st));
  if (dlam)
    HIPCHK(hipMemcpyAsync(dlam, h->dir + h->n, sizeof(double) * h->nlam(), hipMemcpyDeviceToDevice, h->st));
  if (ds) HIPCHK(hipMemcpyAsync(ds, h->ds_w, sizeof(double) * h->ns(), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_step_lengths(qp_handle h, const double* dlam, const double* ds, double gamma,
                          double* alpha_x, double* alpha_lam) {
  if (!h || !dlam || !ds) return QP_ERR_ARG;
  VecArgs v = vec_args(h);
  v.gamma = gamma;
  const int grid = grid_cap(h->ns(), kBlock, kGridMax);
  HIPCHK(launch_ratio_given(v, dlam, ds, grid, h->st));
  HIPCHK(launch_finish_ratio(v, 0, grid, h->st));
  CHK(read_back(h));
  if (alpha_x) *alpha_x = h->hsc[S_ALPHA_X];
  if (alpha_lam) *alpha_lam = h->hsc[S_ALPHA_L];
  return QP_OK;
}

qp_status qp_take_step(qp_handle h, const double* dx, const double* dlam, const double* ds,
                       double alpha_x, double alpha_lam) {
  if (!h || !dx || !dlam || !ds) return QP_ERR_ARG;
  VecArgs v = vec_args(h);
  HIPCHK(launch_update(v, dx, dlam, ds, nullptr, alpha_x, alpha_lam,
                       grid_cap(h->nlam(), kBlock, kGridMax), h->st));
  h->res_valid = h->sys_valid = false;
  h->solved = false;
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

// Mehrotra rule: lam^T s over the inequality pairs into sc[S_MU_CUR] and the
// count of pairs into sc[S_NPAIRS], or, with the predictor's direction,
// its value after the affine steps (alphas in sc) into sc[S_MU_AFF]; read back.
static qp_status mpc_sums(qp_handle h, const double* dlam, const double* ds) {
  VecArgs v = vec_args(h);
  const int grid = grid_cap(h->ns(), kBlock, kGridMax);
  double* P = h->part;
  HIPCHK(launch_compl(v, dlam, ds, P + P_CMP0 * kGridMax, P + P_CMP1 * kGridMax,
                      P + P_CMP2 * kGridMax, grid, h->st));
  HIPCHK(launch_finish_sum(P + P_CMP0 * kGridMax, grid, h->sc + S_MU_CUR, h->st));
  HIPCHK(launch_finish_sum(P + (dlam ? P_CMP1 : P_CMP2) * kGridMax, grid,
                           h->sc + (dlam ? S_MU_AFF : S_NPAIRS), h->st));
  return read_back(h);
}

// Algorithm 1 with the Mehrotra predictor-corrector rule (ipm_options.mu_rule):
// per iteration a predictor and a corrector solve of eq. (9) with one K.
static qp_status run_mpc(qp_handle h, const ipm_options& opt, const pcg_options& po, double np,
                         ipm_info* info, double* pcg_ms, bool* converged, int* iters) {
  const double tol = opt.mu_tol / opt.mu_div;
  if (!h->dlam_aff) CHK(dalloc_t(h, &h->dlam_aff, h->nlam()));
  if (!h->ds_aff) CHK(dalloc_t(h, &h->ds_aff, h->ns()));
  const int gv = grid_cap(h->ns(), kBlock, kGridMax);
  double mu = h->hsc[S_MU_CUR] / np;
  h->tau_on = true;
  int it = 0;
  *converged = false;
  for (it = 1; it <= opt.max_iter; ++it) {
    // predictor: complementarity target 0, penalty mu
    h->mu = mu;
    h->tau = 0.0;
    h->res_valid = h->sys_valid = false;
    CHK(prepare(h));
    auto tp = std::chrono::steady_clock::now();
    pcg_info pa{};
    CHK(run_pcg(h, h->rhs, h->dir, po, &pa));
    *pcg_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
    CHK(run_recover(h, 1.0));
    HIPCHK(launch_copy(h->dir + h->n, h->dlam_aff, h->nlam(), 1.0, h->st));
    HIPCHK(launch_copy(h->ds_w, h->ds_aff, h->ns(), 1.0, h->st));
    CHK(mpc_sums(h, h->dlam_aff, h->ds_aff));
    const double mu_aff = h->hsc[S_MU_AFF] / np;
    const double sigma = std::min(1.0, std::pow(mu_aff / mu, 3.0));
    // corrector: target max(sigma mu, tol / 2), second-order term, same K
    h->tau = std::max(sigma * mu, 0.5 * tol);
    CHK(run_residuals(h));
    VecArgs v = vec_args(h);
    HIPCHK(launch_second_order(v, h->res, h->dlam_aff, h->ds_aff, gv, h->st));
    CHK(run_system(h));
    tp = std::chrono::steady_clock::now();
    pcg_info pc{};
    CHK(run_pcg(h, h->rhs, h->dir, po, &pc));
    *pcg_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
    for (const pcg_info* pi : {&pa, &pc}) {
      info->total_cg_iters += pi->iterations;
      if (!pi->converged) info->cg_maxiter_hits++;
      if (pi->escalated) info->cg_escalations++;
    }
    CHK(run_recover(h, opt.gamma));
    v = vec_args(h);
    HIPCHK(launch_update(v, h->dir, h->dir + h->n, h->ds_w, h->sc + S_ALPHA_X, 0.0, 0.0,
                         grid_cap(h->nlam(), kBlock, kGridMax), h->st));
    h->res_valid = h->sys_valid = false;
    // the new point: mu, and its residuals for that mu (target and penalty),
    // as Algorithm 1 measures them; the stop test uses their primal and dual part
    CHK(mpc_sums(h, nullptr, nullptr));
    const double mu_new = h->hsc[S_MU_CUR] / np;
    h->mu = mu_new;
    h->tau = mu_new;
    CHK(run_residuals(h));
    CHK(read_back(h));
    const double nr = h->hsc[S_NORM], co = h->hsc[S_COMPL];
    if (!std::isfinite(nr) || !std::isfinite(mu_new)) {
      h->tau_on = false;
      h->err = "residual norm is not finite";
      return QP_ERR_NUMERIC;
    }
    const double pd = std::sqrt(std::max(0.0, nr * nr - co * co));
    const int li = it - 1;
    if (li < opt.log_capacity) {
      if (opt.log_mu) opt.log_mu[li] = mu;
      if (opt.log_sigma) opt.log_sigma[li] = sigma;
      if (opt.log_rnorm) opt.log_rnorm[li] = nr;
      if (opt.log_primal) opt.log_primal[li] = h->hsc[S_PRIMAL];
      if (opt.log_dual) opt.log_dual[li] = h->hsc[S_DUAL];
      if (opt.log_compl) opt.log_compl[li] = co;
      if (opt.log_alpha_x) opt.log_alpha_x[li] = h->hsc[S_ALPHA_X];
      if (opt.log_alpha_lam) opt.log_alpha_lam[li] = h->hsc[S_ALPHA_L];
      if (opt.log_cg_iters) opt.log_cg_iters[li] = pa.iterations + pc.iterations;
      if (opt.log_cg_relres) opt.log_cg_relres[li] = pc.rel_residual;
      if (opt.log_kappa)
        opt.log_kappa[li] = pa.lambda_min > 0.0 ? pa.lambda_max / pa.lambda_min : 0.0;
    }
    info->rnorm = nr;
    info->primal = h->hsc[S_PRIMAL];
    info->dual = h->hsc[S_DUAL];
    info->compl_ = co;
    mu = mu_new;
    if (mu < tol && pd < tol) {
      *converged = true;
      break;
    }
  }
  h->tau_on = false;
  h->mu = mu;
  h->res_valid = h->sys_valid = false;
  *iters = *converged ? it : opt.max_iter;
  return QP_OK;
}

qp_status ipm_solve(qp_handle h, const ipm_options* o, double* x, double* lam, double* s,
                    ipm_info* info) {
  if (!h || !info) return QP_ERR_ARG;
  ipm_options opt;
  qp_default_ipm_options(&opt);
  if (o) opt = *o;
  const pcg_options po = pcg_opts_or_default(&opt.pcg);
  if (!(opt.gamma > 0.0 && opt.gamma < 1.0) || !(opt.mu0 > 0.0) || !(opt.mu_div > 1.0) ||
      opt.max_iter < 1 || (opt.mu_rule != QP_MU_PAPER && opt.mu_rule != QP_MU_MEHROTRA)) {
    h->err = "invalid ipm_options";
    return QP_ERR_ARG;
  }
  std::memset(info, 0, sizeof(*info));
  HIPCHK(hipStreamSynchronize(h->st));
  const auto t0 = std::chrono::steady_clock::now();
  double pcg_ms = 0.0;
  if (!opt.warm_start) CHK(run_init_state(h, opt.mu0));
  h->res_valid = h->sys_valid = false;
  h->solved = false;
  int it = 0;
  bool converged = false;
  bool mpc_done = false;
  int mpc_iters = 0;
  if (opt.mu_rule == QP_MU_MEHROTRA) {
    CHK(mpc_sums(h, nullptr, nullptr));
    const double np = h->hsc[S_NPAIRS];
    if (np > 0.0) {
      // with no inequality pairs there is no complementarity: the paper's rule
      CHK(run_mpc(h, opt, po, np, info, &pcg_ms, &converged, &mpc_iters));
      mpc_done = true;
    }
  }
  for (it = 1; !mpc_done && it <= opt.max_iter; ++it) {
    CHK(prepare(h));
    const auto tp = std::chrono::steady_clock::now();
    pcg_info pi{};
    CHK(run_pcg(h, h->rhs, h->dir, po, &pi));
    pcg_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
    info->total_cg_iters += pi.iterations;
    if (!pi.converged) info->cg_maxiter_hits++;
    if (pi.escalated) info->cg_escalations++;
    double kappa_plain = 0.0;
    if (opt.log_kappa_plain && it - 1 < opt.log_capacity) {
      // the spectrum of K itself (Section 5.3), from plain CG on the same system
      if (!h->kap_sol) CHK(dalloc_t(h, &h->kap_sol, h->N()));
      pcg_options pp = po;
      pp.no_precond = 1;
      pp.spectrum = 1;
      pcg_info pk{};
      CHK(run_pcg(h, h->rhs, h->kap_sol, pp, &pk));
      kappa_plain = pk.lambda_min > 0.0 ? pk.lambda_max / pk.lambda_min : 0.0;
    }
    CHK(run_recover(h, opt.gamma));
    VecArgs v = vec_args(h);
    HIPCHK(launch_update(v, h->dir, h->dir + h->n, h->ds_w, h->sc + S_ALPHA_X, 0.0, 0.0,
                         grid_cap(h->nlam(), kBlock, kGridMax), h->st));
    h->res_valid = h->sys_valid = false;
    CHK(run_residuals(h));
    CHK(read_back(h));
    const double nr = h->hsc[S_NORM];
    if (!std::isfinite(nr)) {
      h->err = "residual norm is not finite";
      return QP_ERR_NUMERIC;
    }
    const int li = it - 1;
    if (li < opt.log_capacity) {
      if (opt.log_mu) opt.log_mu[li] = h->mu;
      if (opt.log_rnorm) opt.log_rnorm[li] = nr;
      if (opt.log_primal) opt.log_primal[li] = h->hsc[S_PRIMAL];
      if (opt.log_dual) opt.log_dual[li] = h->hsc[S_DUAL];
      if (opt.log_compl) opt.log_compl[li] = h->hsc[S_COMPL];
      if (opt.log_alpha_x) opt.log_alpha_x[li] = h->hsc[S_ALPHA_X];
      if (opt.log_alpha_lam) opt.log_alpha_lam[li] = h->hsc[S_ALPHA_L];
      if (opt.log_cg_iters) opt.log_cg_iters[li] = pi.iterations;
      if (opt.log_cg_relres) opt.log_cg_relres[li] = pi.rel_residual;
      if (opt.log_kappa)
        opt.log_kappa[li] = pi.lambda_min > 0.0 ? pi.lambda_max / pi.lambda_min : 0.0;
      if (opt.log_kappa_plain) opt.log_kappa_plain[li] = kappa_plain;
    }
    info->rnorm = nr;
    info->primal = h->hsc[S_PRIMAL];
    info->dual = h->hsc[S_DUAL];
    info->compl_ = h->hsc[S_COMPL];
    if (nr < h->mu) {
      if (h->mu < opt.mu_tol) {
        converged = true;
        break;
      }
      h->mu = h->mu / opt.mu_div;
      h->res_valid = h->sys_valid = false;
    }
  }
  if (mpc_done) info->iterations = mpc_iters;
  else info->iterations = converged ? it : opt.max_iter;
  info->result = converged ? QP_IPM_CONVERGED : QP_IPM_MAX_ITER;
  info->mu_final = h->mu;
  CHK(run_objective(h, &info->objective));
  if (x) HIPCHK(hipMemcpyAsync(x, h->x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->st));
  if (lam) HIPCHK(hipMemcpyAsync(lam, h->lam, sizeof(double) * h->nlam(), hipMemcpyDeviceToDevice, h->st));
  if (s) HIPCHK(hipMemcpyAsync(s, h->s, sizeof(double) * h->ns(), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  info->pcg_time_ms = pcg_ms;
  h->solved = true;
  return QP_OK;
}

qp_status qp_backward(qp_handle h, const double* grad_x, double* grad_c, double* grad_lA,
                      double* grad_uA, double* grad_b, double* grad_w, const pcg_options* o,
                      pcg_info* info) {
  if (!h || !grad_x) return QP_ERR_ARG;
  if (!h->solved) {
    h->err = "qp_backward needs a completed ipm_solve on this handle";
    return QP_ERR_STATE;
  }
  if (grad_w && h->p_rows == 0) {
    h->err = "grad_w needs a P^T W P Hessian";
    return QP_ERR_ARG;
  }
  CHK(prepare(h));
  // adjoint right-hand side (grad_x, 0)
  double* arhs = h->arhs;
  HIPCHK(launch_fill(arhs, h->N(), 0.0, h->st));
  HIPCHK(launch_copy(grad_x, arhs, h->n, 1.0, h->st));
  pcg_options po = pcg_opts_or_default(o);
  if (!o) po.tol = 1e-10;
  double* usol = h->dir;  // the direction buffer is free after the solve
  pcg_info inf{};
  qp_status s = run_pcg(h, arhs, usol, po, &inf);
  if (info) *info = inf;
  if (s != QP_OK) return s;
  HIPCHK(launch_grad_out(h->n, h->m, h->me, usol, h->lA, h->uA, grad_c, grad_lA, grad_uA, grad_b, h->st));
  if (grad_w) {
    RowArgs a = row_args(h, false);
    a.r0 = 0; a.r1 = h->p_rows; a.v = usol; a.v2 = h->x; a.gw = grad_w;
    HIPCHK(launch_rowpass(R_GRADW, VK_F64, h->lpr_r, a, h->g_r, h->st));
  }
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_update_data(qp_handle h, const double* c, const double* lA, const double* uA,
                         const double* b, const double* w) {
  if (!h) return QP_ERR_ARG;
  if (w && h->p_rows == 0) {
    h->err = "weights apply to a P^T W P Hessian only";
    return QP_ERR_ARG;
  }
  if (c) HIPCHK(hipMemcpyAsync(h->c, c, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->st));
  if (lA && h->m) HIPCHK(hipMemcpyAsync(h->lA, lA, sizeof(double) * h->m, hipMemcpyDeviceToDevice, h->st));
  if (uA && h->m) HIPCHK(hipMemcpyAsync(h->uA, uA, sizeof(double) * h->m, hipMemcpyDeviceToDevice, h->st));
  if (b && h->me) HIPCHK(hipMemcpyAsync(h->b, b, sizeof(double) * h->me, hipMemcpyDeviceToDevice, h->st));
  if (w) HIPCHK(hipMemcpyAsync(h->pw, w, sizeof(double) * h->p_rows, hipMemcpyDeviceToDevice, h->st));
  CHK(derive_constants(h));
  h->res_valid = h->sys_valid = false;
  h->solved = false;
  HIPCHK(hipStreamSynchronize(h->st));
  return QP_OK;
}

qp_status qp_profile_begin(qp_handle h, int32_t max_launches, int32_t every) {
  if (!h || max_launches < 1 || every < 1) return QP_ERR_ARG;
  for (int c = 0; c < QP_PROF_COUNT; ++c) {
    for (hipEvent_t e : h->prof.ev[c]) (void)hipEventDestroy(e);
    h->prof.ev[c].assign(2 * (size_t)max_launches, nullptr);
    for (auto& e : h->prof.ev[c]) HIPCHK(hipEventCreate(&e));
    h->prof.used[c] = 0;
    h->prof.seen[c] = 0;
  }
  h->prof.cap = max_launches;
  h->prof.every = every;
  h->prof.on = true;
  return QP_OK;
}

qp_status qp_profile_end(qp_handle h, int64_t* launches, double* total_ms, int64_t* dispatches) {
  if (!h || !h->prof.on) return QP_ERR_STATE;
  HIPCHK(hipStreamSynchronize(h->st));
  for (int c = 0; c < QP_PROF_COUNT; ++c) {
    double tot = 0.0;
    for (int i = 0; i < h->prof.used[c]; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, h->prof.ev[c][2 * i], h->prof.ev[c][2 * i + 1]));
      tot += ms;
    }
    if (launches) launches[c] = h->prof.used[c];
    if (total_ms) total_ms[c] = tot;
    if (dispatches) dispatches[c] = h->prof.seen[c];
    for (hipEvent_t e : h->prof.ev[c]) (void)hipEventDestroy(e);
    h->prof.ev[c].clear();
    h->prof.used[c] = 0;
    h->prof.seen[c] = 0;
  }
  h->prof.on = false;
  h->prof.cap = 0;
  return QP_OK;
}

qp_status qp_operator_bytes(qp_handle h, int64_t* row_bytes, int64_t* col_bytes,
                            int64_t* dense_bytes, int64_t* row_nnz, int64_t* col_nnz) {
  if (!h) return QP_ERR_ARG;
  const int64_t vb = h->vk == VK_F64 ? 8 : (h->vk == VK_F32 || h->vk == VK_F32X) ? 4 : 2;
  // bytes of the structures the PCG matvec streams (values, column indices, row pointers)
  auto ck_bytes = [&](const qp_handle_s::Chunked& k) {
    return k.nnz * (vb + 2) + 4 * (int64_t)k.nchunk * (k.nrows + 1);
  };
  if (row_bytes)
    *row_bytes = h->ck_r.on ? ck_bytes(h->ck_r) + (h->fold_a ? 4 * (int64_t)h->p_rows : 0)
                            : h->nnz_rp * (vb + 4) + 4 * (int64_t)(h->nRP + 1);
  if (col_bytes)
    *col_bytes = h->ck_x.on ? ck_bytes(h->ck_x) : h->nnz_xs * (vb + 4) + 12 * (int64_t)h->n + 4;
  if (dense_bytes) *dense_bytes = (int64_t)h->n * h->k * vb;
  if (row_nnz) *row_nnz = h->nnz_rp;
  if (col_nnz) *col_nnz = h->nnz_xs;
  return QP_OK;
}

qp_status qp_graph_stats(qp_handle h, int64_t* captures, int64_t* replays) {
  if (!h) return QP_ERR_ARG;
  if (captures) *captures = h->gr.captures;
  if (replays) *replays = h->gr.replays;
  return QP_OK;
}

qp_status qp_fused_layout(qp_handle h, int32_t* active, int32_t* ranges, int32_t* half_cols,
                          int64_t* stored, int32_t* failed) {
  if (!h) return QP_ERR_ARG;
  if (active) *active = fused_active(h) ? 1 : 0;
  if (ranges) *ranges = h->fz.on ? h->fz.nrange : 0;
  if (half_cols) *half_cols = h->fz.on ? h->fz.half : 0;
  if (stored) *stored = h->fz.on ? h->fz.stored : 0;
  if (failed) *failed = h->fz.failed ? 1 : 0;
  return QP_OK;
}

qp_status qp_operator_layout(qp_handle h, int32_t* chunks, int32_t* work_items,
                             int32_t* chunk_cols) {
  if (!h) return QP_ERR_ARG;
  const qp_handle_s::Chunked* side[2] = {&h->ck_r, &h->ck_x};
  for (int i = 0; i < 2; ++i) {
    const bool on = side[i]->on;
    if (chunks) chunks[i] = on ? side[i]->nchunk : 0;
    if (work_items) work_items[i] = on ? side[i]->nwork : (i == 0 ? h->g_rmv : h->g_xmv);
    if (chunk_cols) chunk_cols[i] = on ? side[i]->chunk_cols : 0;
  }
  return QP_OK;
}

}  // extern "C"
