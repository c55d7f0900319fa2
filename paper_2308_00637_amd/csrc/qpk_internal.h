// Internal declarations shared by the kernels and the host side of libqpk.
// Layout notes (all float64 unless stated):
//   lam = [e (me) | lA (m) | uA (m) | lx (n) | ux (n)],  s = [lA (m) | uA (m) | lx (n) | ux (n)]
//   K-vector (eq. (9)) = [x (n) | e (me) | lA (m) | uA (m)]
//   residual stack = [rH n | re me | rlA m | ruA m | rlx n | rux n | rc1 m | rc2 m | rc3 n | rc4 n]
// Row-side operator "RP" is one CSR holding the rows of P (H = P^T W P) followed
// by the rows of A.  Column-side operator "XS" holds, for every variable j, three
// consecutive segments: dense-H row j (gathers x), column j of P (gathers the
// per-voxel values u), column j of A (gathers the per-row values wA).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace qpk {

constexpr int kBlock = 256;      // threads per block for every kernel
constexpr int kGridMax = 2048;   // cap on blocks of grid-stride kernels (= partial slots)
constexpr int QP_ERR_NOT_SPD_CODE = -4;   // mirrors qp_status in qpk.h
constexpr int QP_ERR_NUMERIC_CODE = -5;

// Stored value type and accumulation type of the PCG matvec passes.
enum ValKind : int { VK_F64 = 0, VK_F32 = 1, VK_BF16 = 2, VK_F32X = 3, VK_BF16X = 4 };

// Row-side pass modes
enum RowMode : int {
  R_MATVEC = 0,   // P rows: u = w (P_v.v);  A rows: lam-part of K v, wA = w_l - w_u
  R_RESID = 1,    // P rows: u = w (P_v.x);  A rows: r_lA, r_uA, r_c1, r_c2, wA = lam_u - lam_l
  R_RECOVER = 2,  // A rows: ds_lA, ds_uA from dx, ratio-test minima
  R_GRADW = 3,    // P rows: gw_v = -(P_v.a)(P_v.x - d_v)
  R_PU = 4,       // P rows only: u = w (P_v.x)
  R_INIT = 5      // A rows: default starting slacks from t = A_i x
};

// Column-side pass modes
enum ColMode : int {
  X_MATVEC = 0,   // x-part of K v
  X_RESID = 1,    // r_H, r_lx, r_ux, r_c3, r_c4
  X_RHS = 2,      // top of the eq. (9) right-hand side, Jacobi diagonal, Q diagonal
  X_DIAGH = 3,    // diag(P^T W P) + sum_l wd_l U_jl^2 (accumulated into diagH)
  X_CEFF = 4,     // c_eff = c - P^T (w d)
  X_OBJ = 5       // partial sums of x_j (1/2 (Hx)_j + c_j)
};

struct RowArgs {
  int32_t r0, r1;            // RP row range to process
  int32_t p_rows, m, n, me;
  const int32_t* rowptr;
  const int32_t* col;
  const void* val;
  const double* v;           // gathered x-space vector
  const double* v2;          // second gathered vector (R_GRADW: x)
  const double* w;           // P row weights
  const double* d;           // P row targets
  double* u;                 // P row outputs
  double* wA;                // A row outputs
  const double* lA;
  const double* uA;
  const double* vl;          // lam-part of the input K-vector (me + 2m)
  const double* dl;          // D (me + 2m)
  double* yl;                // lam-part of the output K-vector
  const double* lam;
  const double* s;
  double mu;
  double tau;                // complementarity target of R_RESID (mu under the paper's rule)
  const double* res;         // residual stack (R_RECOVER reads r_lA, r_uA)
  double* resw;              // residual stack output (R_RESID)
  const double* dlam;        // R_RECOVER: direction lam (iterate layout)
  double* ds;                // R_RECOVER: slack direction out
  double* part0;             // per-block partials
  double* part1;
  double* gw;                // R_GRADW output
  const int* done;           // optional early-exit flag (PCG)
  int* bump;                 // optional PCG iteration counter to advance
  // R_MATVEC / CE_ROW: also accumulate v_x . (K v)_x into part0 (the column
  // pass then leaves its x-part unsummed; see CgArgs::qpart)
  int32_t xdot;
  const double* qdiag;       // n
  const double* Cm;          // me*n row-major
  const double* we;          // me
  // R_MATVEC / CE_ROW on a blocked row side that holds P alone: per P row,
  // the row of A that repeats it (or -1).  Its A-row epilogue runs on the P
  // row's dot, and u then carries u + wA for the column pass.
  const int32_t* twin;
};

struct ColArgs {
  int32_t n, me, m, p_rows, k;
  const int32_t* rowptr;
  const int32_t* seg1;
  const int32_t* seg2;
  const int32_t* col;
  const void* val;
  int use_hx, use_pt, use_at;
  const double* src_hx;      // n
  const double* src_pt;      // p_rows
  const double* src_at;      // m
  const double* src_at2;     // m (X_RHS: Jacobi weights)
  const void* U;             // n*k (value kind as val)
  const double* g;           // k, already scaled by wd
  const double* Cm;          // me*n row-major, float64
  const double* we;          // me
  const double* v;           // x-space vector for the diagonal term
  const double* qdiag;       // n
  double* y;                 // output x-part
  const double* c;
  const double* h0;
  const double* lam;
  const double* s;
  const double* lx;
  const double* ux;
  double mu;
  double tau;                // complementarity target of X_RESID (mu under the paper's rule)
  double* res;
  const double* res_in;
  double* rhs;
  double* jdiag;
  const double* diagH;
  double* qdiag_out;
  const double* wd;
  const double* w;           // X_DIAGH: P row weights
  double* part0;
  double* part1;
  double* part2;
  const int* done;
  int* bump;
};

// Tall-skinny dense reduction g = U^T v (k columns) and te = C v (me rows).
struct TsArgs {
  int32_t n, k, me;
  const void* U;
  const double* Cm;
  const double* v;
  double* part;              // [grid][k + me]
  int32_t chunk;             // rows per block
  const int* done;
};

// Optional timing of a single dispatch.  With start set, the launcher issues
// the kernel through hipExtLaunchKernelGGL, which ties both events to that
// dispatch alone (no queue gap before or after it is counted).
struct KEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
template <typename F, typename... A>
inline hipError_t launch_ev(const KEvents* ev, F kern, dim3 grid, dim3 block, uint32_t lds,
                            hipStream_t st, A... args) {
  if (ev && ev->start)
    hipExtLaunchKernelGGL(kern, grid, block, lds, st, ev->start, ev->stop, 0u, args...);
  else
    kern<<<grid, block, lds, st>>>(args...);
  return hipGetLastError();
}

// Launchers (defined in qpk_kernels.hip).  lpr: lanes per row (4..64).
hipError_t launch_rowpass(int mode, int vk, int lpr, const RowArgs& a, int grid, hipStream_t st,
                          const KEvents* ev = nullptr);
hipError_t launch_colpass(int mode, int vk, int lpr, const ColArgs& a, int grid, hipStream_t st,
                          const KEvents* ev = nullptr);
hipError_t launch_ts_reduce(int vk, const TsArgs& a, int grid, hipStream_t st,
                            const KEvents* ev = nullptr);

// LDS-staged 2-D blocked passes.  The columns of a CSR operator are cut into
// chunks of kChunkCols; chunk c stores its own CSR (rowptr c*(nrows+1) ...,
// uint16 column offsets within the chunk).  A block takes one work item
// (chunk, first row, end row), copies that chunk of the gathered vector into
// LDS and reduces its rows from there.  With one chunk the row epilogue runs in
// place; otherwise per-chunk partial sums are written and an epilogue kernel
// adds them in chunk order (in a PCG iteration on a single-chunk row side,
// k_cg_update adds the column side's itself).
constexpr int kChunkBlock = 1024;                 // threads per block
constexpr int kChunkCols = 20224;                 // most float64 values per LDS chunk
struct ChunkArgs {
  int32_t nrows, ncols, nchunk;
  int32_t chunk_cols;        // columns per chunk (<= kChunkCols); LDS = 8 * chunk_cols bytes
  const int32_t* work;       // 3 per block: chunk, r0, r1
  const int32_t* rowptr;     // nchunk * (nrows + 1)
  const uint16_t* col;
  const void* val;
  const double* src;         // gathered vector (ncols)
  double* partial;           // nchunk * nrows when nchunk > 1
  int32_t nstored;           // stored entries (with the even-length padding)
  int32_t kv;                // chunk staging: 0 through registers, 1 direct to LDS
  int32_t reverse;           // visit each work item's rows last to first
  int32_t xcd_map;           // runs of consecutive work items per XCD (see k_chunked)
};
constexpr int kKvDefault = 1;
enum ChunkEpi : int { CE_PARTIAL = 0, CE_ROW = 1, CE_COL = 2 };
hipError_t launch_chunked(int epi, int vk, int lpr, const ChunkArgs& c, const RowArgs& ra,
                          const ColArgs& ca, int nwork, hipStream_t st, const KEvents* ev = nullptr);
hipError_t launch_chunk_epilogue_col(const ChunkArgs& c, const ColArgs& ca, int grid, hipStream_t st,
                                     const KEvents* ev = nullptr);
hipError_t launch_chunk_epilogue_row(const ChunkArgs& c, const RowArgs& ra, int grid, hipStream_t st,
                                     const KEvents* ev = nullptr);
hipError_t chunked_set_attributes();

// Fused single-read PCG product for H = P^T W P (see k_fused).  The row
// operator's columns are cut into two halves (half 0: [0, half), half 1:
// [half, ncols)); a pair of blocks per row range, one per half, exchanges the
// half dots of each row through xch.
constexpr int kFusedLpr = 8;                          // lanes per row
constexpr int kFusedOwn = (kChunkBlock / 64) * 3 * (64 / kFusedLpr);   // float64 dots kept in LDS
constexpr int kFusedHalfMax = (163840 - 256 - 8 * kFusedOwn) / 16;    // columns per half
struct FusedArgs {
  int32_t nrows, ncols;      // rows of the row operator, n
  int32_t half;              // columns of half 0 (even, >= ncols - half)
  int32_t nrange;            // row ranges (2 nrange blocks)
  const int32_t* range;      // nrange + 1 row boundaries
  const int32_t* rowptr;     // 2 * (nrows + 1): half 0's CSR, then half 1's
  const uint16_t* col;       // column offsets within the half
  const void* val;
  int32_t nstored;
  const double* src;         // gathered x-space vector (ncols)
  const int32_t* rowinfo;    // per row: index of the row of A it carries | bit 30 finite
                             // lower side | bit 29 finite upper side, or -1
  double* xch;               // 2 parities x 2 halves x nrows half dots (all bits set = empty)
  int* abort;                // sticky: a wait timed out, the product is invalid
  unsigned long long epoch;  // launch count (its parity picks the exchange slots)
  int32_t spin_max;          // bound on a wait's polls
  double* ypart;             // nrange * ncols: each range's x-part of K v
};
hipError_t launch_fused(int vk, const FusedArgs& f, const RowArgs& ra, hipStream_t st,
                        const KEvents* ev = nullptr);
hipError_t fused_set_attributes();

}  // namespace qpk

namespace qpk {

// Partial-sum regions (each kGridMax doubles) in one device array.
enum PartRegion : int {
  P_DOT_R = 0, P_DOT_X, P_DOT_TS, P_RZ0, P_RZ1, P_RR, P_RR0,
  P_NR_PRIMAL, P_NR_COMPL, P_NX_DUAL, P_NX_PRIMAL, P_NX_COMPL, P_NTS_RE,
  P_MIN_S_R, P_MIN_L_R, P_MIN_S_X, P_MIN_L_X, P_OBJ, P_CHK, P_CMP0, P_CMP1, P_CMP2, P_COUNT
};

// Device scalars (double) and flags (int).
enum Scalar : int {
  S_ALPHA_X = 0, S_ALPHA_L, S_NORM, S_PRIMAL, S_DUAL, S_COMPL, S_RHSNORM,
  S_OBJ, S_RELRES, S_RECUR,
  S_MU_CUR, S_MU_AFF, S_NPAIRS,   // Mehrotra rule: lam^T s, its value after the affine steps, N_c
  S_COUNT
};
enum Flag : int { F_DONE = 0, F_CNT, F_STATUS, F_ITERS, F_BAD, F_FUSEFAIL, F_COUNT };

// Single-block finisher of the tall-skinny reduction.
enum TsMode : int { TS_MATVEC = 0, TS_RESID = 1, TS_GONLY = 2 };
struct TsFinishArgs {
  int32_t n, k, me, grid;
  const double* part;        // [grid][k+me]
  const double* wd;
  double* g;                 // k
  double* te;                // me (C v)
  double* we;                // me
  const double* vl;          // TS_MATVEC: lam-part of input (e entries first)
  double* yl;                // TS_MATVEC: lam-part of output
  const double* b;
  const double* lam;
  double mu;
  double* res;               // TS_RESID: residual stack
  double* partout;           // one value
  const int* done;
};
hipError_t launch_ts_finish(int mode, const TsFinishArgs& a, hipStream_t st);

struct VecArgs {
  int32_t n, m, me, N;       // N = n + me + 2m
  double* x;
  double* lam;
  double* s;
  const double* lA;
  const double* uA;
  const double* lx;
  const double* ux;
  const double* b;
  double mu;
  const double* res;
  double* rhs;
  double* jdiag;
  double* dl;
  double* wA;
  double* jw;
  double* we;
  const double* dx;
  const double* dlam;
  double* ds;
  double* dlam_w;
  double gamma;
  double* part;              // partial base (P_COUNT regions)
  double* sc;
  int* fl;
  int g_r, g_x;              // grids of the row/col passes (partial counts)
};
hipError_t launch_rhs_lam(const VecArgs& a, hipStream_t st);
hipError_t launch_recover_x(const VecArgs& a, int grid, hipStream_t st);
hipError_t launch_finish_ratio(const VecArgs& a, int g_r, int g_x, hipStream_t st);
hipError_t launch_finish_norms(const VecArgs& a, int g_r, int g_x, hipStream_t st);
hipError_t launch_update(const VecArgs& a, const double* dx, const double* dlam,
                         const double* ds, const double* alpha_dev, double ax, double al,
                         int grid, hipStream_t st);
hipError_t launch_init_x(const VecArgs& a, int grid, hipStream_t st);
hipError_t launch_check_state(const VecArgs& a, int grid, hipStream_t st);
hipError_t launch_finish_sum(const double* part, int count, double* out, hipStream_t st);

// PCG kernels
struct CgArgs {
  int32_t N, n;
  double* x;
  double* r;
  double* z;
  double* p;
  double* q;
  const double* rhs;
  const double* jdiag;
  double* part;              // partial base
  int* fl;
  double* sc;
  int g_vec;                 // grid of the vector kernels
  int g_r, g_x, has_ts;      // partial counts of the matvec passes
  double tol;
  int maxit;
  // Column epilogue folded into the update: when qpart is set, the x-part of
  // q is summed here from the column pass's per-chunk partials (nchunk x n),
  // plus the equality and diagonal terms, instead of being read from q.
  const double* qpart;
  int nchunk, me;
  const double* qdiag;
  const double* Cm;
  const double* we;
  double* coef;              // optional: alpha_k at 2k, beta_k at 2k + 1 (Lanczos)
};
hipError_t launch_cg_init(const CgArgs& a, hipStream_t st);
hipError_t launch_cg_update(const CgArgs& a, hipStream_t st, const KEvents* ev = nullptr);
hipError_t launch_cg_pupdate(const CgArgs& a, hipStream_t st, const KEvents* ev = nullptr);
hipError_t launch_cg_restart(const CgArgs& a, const double* kx, int resume, hipStream_t st);

// Backward: gradient outputs from the adjoint solution u (K-vector layout).
hipError_t launch_grad_out(int n, int m, int me, const double* u, const double* lA,
                           const double* uA, double* gc, double* glA, double* guA,
                           double* gb, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int64_t n, double scale, hipStream_t st);
hipError_t launch_fill(double* dst, int64_t n, double v, hipStream_t st);
hipError_t launch_sqdiff(const double* a, const double* b, int64_t n, double* part, int grid,
                         hipStream_t st);
hipError_t launch_ratio_given(const VecArgs& a, const double* dlam, const double* ds, int grid,
                              hipStream_t st);
// Mehrotra rule: per-block sums of lam^T s (part0), of (lam + al dlam)^T
// (s + ax ds) with the ratio test's alphas from sc (part1, when dlam is set)
// and of the count of finite sides (part2); and the corrector's
// complementarity residuals r_c += dlam * ds.
hipError_t launch_compl(const VecArgs& a, const double* dlam, const double* ds, double* part0,
                        double* part1, double* part2, int grid, hipStream_t st);
hipError_t launch_second_order(const VecArgs& a, double* res, const double* dlam, const double* ds,
                               int grid, hipStream_t st);

}  // namespace qpk
