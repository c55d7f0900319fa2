// Batched solving of many independent dense QPs in one persistent launch.
//
// Every workgroup (1024 threads) takes instances from a queue (largest work
// first) and runs the whole of Algorithm 1 (Section 3.2) for each on the
// device: residuals (eq. 3), the eq. 9 right-hand side and Jacobi diagonal,
// Jacobi PCG on eq. 9 (Section 3.1; tolerance on the unpreconditioned relative
// residual, Section 5.1), recovery of the eliminated unknowns (eq. 7), the
// ratio test (eq. 10), the update and the barrier rule.  Workgroups never wait
// for each other: the only cross-workgroup state is the queue counter, so every
// wave reaches the exit when the queue is empty.  The same kernel serves a
// single small problem, where one launch replaces thousands of short ones.
//
// Supported per instance: H dense (n x n) or H = diag(h0) + U diag(wd) U^T
// (U n x k); general rows lA <= A x <= uA with A dense (m x n, m may be 0);
// variable bounds; no equality rows.  A, H and U are stored in float64 or
// float32; vectors, accumulation and all reductions are float64.
#include "qpk_internal.h"
#include "../../include/qpk.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace qpk {

constexpr int kBB = 1024;            // threads per workgroup
constexpr int kBW = kBB / 64;        // waves per workgroup

struct BInst {
  int32_t n, m, k, hkind;            // hkind: 0 dense H, 1 low rank
  const void* A;                     // m x n row-major, in the operator precision
  const void* H;                     // n x n (or U, n x k) row-major, likewise
  int64_t v_off;                     // offset of the instance's float64 block
};

// Float64 block of one instance (me = 0; N = n + 2m).
struct BLayout {
  int64_t c, h0, wd, lA, uA, lx, ux, diagH, x, lam, s, res, rhs, jd, dl, qd, wv, jw, t, g, gw,
      r, z, p, q, sol, ds, ya, yh, total;
  __host__ __device__ BLayout(int64_t n, int64_t m, int64_t k) {
    const int64_t N = n + 2 * m, nl = 2 * m + 2 * n;
    int64_t o = 0;
    c = o; o += n;   h0 = o; o += n;   wd = o; o += k;   lA = o; o += m;   uA = o; o += m;
    lx = o; o += n;  ux = o; o += n;   diagH = o; o += n;
    x = o; o += n;   lam = o; o += nl; s = o; o += nl;
    res = o; o += 5 * n + 4 * m;
    rhs = o; o += N; jd = o; o += N;  dl = o; o += 2 * m; qd = o; o += n;
    wv = o; o += m;  jw = o; o += m;  t = o; o += m;      g = o; o += k;  gw = o; o += k;
    r = o; o += N;   z = o; o += N;   p = o; o += N;      q = o; o += N;
    sol = o; o += n + nl;             ds = o; o += nl;    ya = o; o += n; yh = o; o += n;
    total = o;
  }
};

struct BOpts {
  double gamma, mu0, mu_tol, mu_div, cg_tol;
  int32_t max_iter, cg_maxit;
};

// Per-instance result (float64 fields, then counters).
struct BResult {
  double mu_final, rnorm, primal, dual, compl_, objective;
  int32_t status, iterations, cg_hits, pad;
  int64_t total_cg;
};

template <typename T>
struct BArgs {
  const BInst* inst;
  const int32_t* order;
  int32_t count;
  int32_t* next;
  double* vec;
  BResult* out;
  BOpts o;
};

__device__ __forceinline__ bool blo(double l) { return l > -INFINITY; }
__device__ __forceinline__ bool bhi(double u) { return u < INFINITY; }

// Reductions over the workgroup; the result is returned to every thread.
__device__ __forceinline__ double wg_sum(double v) {
  __shared__ double sh[kBW];
  __shared__ double res;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kBW; ++i) s += sh[i];
    res = s;
  }
  __syncthreads();
  const double r = res;
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wg_min(double v) {
  __shared__ double sh[kBW];
  __shared__ double res;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = INFINITY;
#pragma unroll
    for (int i = 0; i < kBW; ++i) s = fmin(s, sh[i]);
    res = s;
  }
  __syncthreads();
  const double r = res;
  __syncthreads();
  return r;
}

// out[r] = sum_c M[r][c] * v[c] (SQ: M^2), one wave per row.
template <bool SQ, typename T>
__device__ __forceinline__ void rowdots(const T* __restrict__ M, int R, int Cn,
                                        const double* __restrict__ v, double* __restrict__ out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = w; r < R; r += kBW) {
    const T* row = M + static_cast<int64_t>(r) * Cn;
    double acc = 0.0;
    for (int c = lane; c < Cn; c += 64) {
      const double a = static_cast<double>(row[c]);
      acc += (SQ ? a * a : a) * v[c];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) out[r] = acc;
  }
}

// out[c] = sum_r M[r][c] * w[r] (SQ: M^2): 256-column tiles, four row groups
// per tile, combined in LDS in group order.
template <bool SQ, typename T>
__device__ __forceinline__ void coldots(const T* __restrict__ M, int R, int Cn,
                                        const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double red[kBB];
  const int cc = threadIdx.x & 255, rg = threadIdx.x >> 8;
  for (int c0 = 0; c0 < Cn; c0 += 256) {
    const int c = c0 + cc;
    double acc = 0.0;
    if (c < Cn) {
      for (int r = rg; r < R; r += 4) {
        const double a = static_cast<double>(M[static_cast<int64_t>(r) * Cn + c]);
        acc += (SQ ? a * a : a) * w[r];
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (rg == 0 && c < Cn) out[c] = red[cc] + red[256 + cc] + red[512 + cc] + red[768 + cc];
    __syncthreads();
  }
}

template <typename T>
struct Inst {
  int n, m, k, hk;
  const T* A;
  const T* H;  // dense H or U
  double* v;
  BLayout L;
  __device__ Inst(const BInst& bi, double* vec)
      : n(bi.n), m(bi.m), k(bi.k), hk(bi.hkind), A(static_cast<const T*>(bi.A)),
        H(static_cast<const T*>(bi.H)),
        v(vec + bi.v_off), L(bi.n, bi.m, bi.k) {}
  __device__ double* P(int64_t off) const { return v + off; }
};

// y = H x into ya (dense: row dots; low rank: h0 x + U (wd * (U^T x))).
template <typename T>
__device__ __forceinline__ void hess_apply(const Inst<T>& I, const double* x, double* y) {
  double* g = I.P(I.L.g);
  double* gw = I.P(I.L.gw);
  if (I.hk == 0) {
    rowdots<false>(I.H, I.n, I.n, x, y);
    __syncthreads();
    return;
  }
  coldots<false>(I.H, I.n, I.k, x, g);
  __syncthreads();
  for (int l = threadIdx.x; l < I.k; l += kBB) gw[l] = I.P(I.L.wd)[l] * g[l];
  __syncthreads();
  rowdots<false>(I.H, I.n, I.k, gw, y);
  __syncthreads();
  const double* h0 = I.P(I.L.h0);
  for (int j = threadIdx.x; j < I.n; j += kBB) y[j] += h0[j] * x[j];
  __syncthreads();
}

// Residual stack (eq. 3 with the bound rows) and its norms; returns
// {stacked, primal, dual, compl}.
template <typename T>
__device__ __noinline__ void residuals(const BInst* bi, double* vec, double mu,
                                    double* nrm) {
  const Inst<T> I(*bi, vec);
  const int n = I.n, m = I.m;
  const double *x = I.P(I.L.x), *lam = I.P(I.L.lam), *s = I.P(I.L.s);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  double *res = I.P(I.L.res), *t = I.P(I.L.t), *wv = I.P(I.L.wv), *ya = I.P(I.L.ya), *yh = I.P(I.L.yh);
  const int64_t oH = 0, olA = n, ouA = n + m, olx = n + 2 * m, oux = 2 * n + 2 * m,
                oc1 = 3 * n + 2 * m, oc2 = 3 * n + 3 * m, oc3 = 3 * n + 4 * m, oc4 = 4 * n + 4 * m;
  if (m > 0) rowdots<false>(I.A, m, n, x, t);
  __syncthreads();
  double pr = 0.0, du = 0.0, co = 0.0;
  for (int i = threadIdx.x; i < m; i += kBB) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double ll = lam[i], lu = lam[m + i], sl = s[i], su = s[m + i];
    const double rl = hl ? t[i] - sl - lA[i] : 0.0;
    const double ru = hu ? -t[i] - su + uA[i] : 0.0;
    const double c1 = hl ? ll * sl - mu : 0.0;
    const double c2 = hu ? lu * su - mu : 0.0;
    res[olA + i] = rl; res[ouA + i] = ru; res[oc1 + i] = c1; res[oc2 + i] = c2;
    wv[i] = (hu ? lu : 0.0) - (hl ? ll : 0.0);
    pr += rl * rl + ru * ru;
    co += c1 * c1 + c2 * c2;
  }
  __syncthreads();
  if (m > 0) coldots<false>(I.A, m, n, wv, ya);
  __syncthreads();
  hess_apply(I, x, yh);
  const double* c = I.P(I.L.c);
  for (int j = threadIdx.x; j < n; j += kBB) {
    const bool hl = blo(lx[j]), hu = bhi(ux[j]);
    const double llx = hl ? lam[2 * m + j] : 0.0, lux = hu ? lam[2 * m + n + j] : 0.0;
    const double slx = s[2 * m + j], sux = s[2 * m + n + j];
    const double rH = yh[j] + c[j] + (m > 0 ? ya[j] : 0.0) - llx + lux;
    const double rlx = hl ? x[j] - slx - lx[j] : 0.0;
    const double rux = hu ? -x[j] - sux + ux[j] : 0.0;
    const double c3 = hl ? llx * slx - mu : 0.0;
    const double c4 = hu ? lux * sux - mu : 0.0;
    res[oH + j] = rH; res[olx + j] = rlx; res[oux + j] = rux; res[oc3 + j] = c3; res[oc4 + j] = c4;
    du += rH * rH;
    pr += rlx * rlx + rux * rux;
    co += c3 * c3 + c4 * c4;
  }
  pr = wg_sum(pr);
  du = wg_sum(du);
  co = wg_sum(co);
  nrm[0] = sqrt(pr + du + co);
  nrm[1] = sqrt(pr);
  nrm[2] = sqrt(du);
  nrm[3] = sqrt(co);
}

// D, the eq. 9 right-hand side, diag(K) and Q's diagonal (eqs. 8, 9).
template <typename T>
__device__ __noinline__ void newton_system(const BInst* bi, double* vec, double mu) {
  const Inst<T> I(*bi, vec);
  const int n = I.n, m = I.m;
  const double *lam = I.P(I.L.lam), *s = I.P(I.L.s), *res = I.P(I.L.res);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  double *rhs = I.P(I.L.rhs), *jd = I.P(I.L.jd), *dl = I.P(I.L.dl), *qd = I.P(I.L.qd);
  double *wv = I.P(I.L.wv), *jw = I.P(I.L.jw), *ya = I.P(I.L.ya), *yh = I.P(I.L.yh);
  const int64_t olA = n, ouA = n + m, olx = n + 2 * m, oux = 2 * n + 2 * m,
                oc1 = 3 * n + 2 * m, oc2 = 3 * n + 3 * m, oc3 = 3 * n + 4 * m, oc4 = 4 * n + 4 * m;
  for (int i = threadIdx.x; i < m; i += kBB) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double ll = lam[i], lu = lam[m + i];
    const double dL = hl ? s[i] / ll : 1.0, dU = hu ? s[m + i] / lu : 1.0;
    const double r2L = hl ? -res[olA + i] - res[oc1 + i] / ll : 0.0;
    const double r2U = hu ? -res[ouA + i] - res[oc2 + i] / lu : 0.0;
    rhs[n + i] = r2L; rhs[n + m + i] = r2U;
    jd[n + i] = dL; jd[n + m + i] = dU;
    dl[i] = dL; dl[m + i] = dU;
    wv[i] = (hl ? 2.0 * r2L / dL : 0.0) - (hu ? 2.0 * r2U / dU : 0.0);
    jw[i] = (hl ? 2.0 / dL : 0.0) + (hu ? 2.0 / dU : 0.0);
  }
  __syncthreads();
  if (m > 0) {
    coldots<false>(I.A, m, n, wv, ya);
    coldots<true>(I.A, m, n, jw, yh);
  }
  __syncthreads();
  const double *diagH = I.P(I.L.diagH), *h0 = I.P(I.L.h0);
  for (int j = threadIdx.x; j < n; j += kBB) {
    const bool hl = blo(lx[j]), hu = bhi(ux[j]);
    const double llx = hl ? lam[2 * m + j] : 0.0, lux = hu ? lam[2 * m + n + j] : 0.0;
    const double slx = hl ? s[2 * m + j] : 1.0, sux = hu ? s[2 * m + n + j] : 1.0;
    const double qb = (hl ? llx / slx : 0.0) + (hu ? lux / sux : 0.0);
    double r1 = -res[j];
    if (hl) r1 += -res[oc3 + j] / slx - llx / slx * res[olx + j];
    if (hu) r1 += res[oc4 + j] / sux + lux / sux * res[oux + j];
    rhs[j] = r1 + (m > 0 ? ya[j] : 0.0);
    jd[j] = diagH[j] + qb + (m > 0 ? yh[j] : 0.0);
    qd[j] = (I.hk == 1 ? h0[j] : 0.0) + qb;
  }
  __syncthreads();
}

// q = K p (eq. 9, matrix-free); returns p . q.
template <typename T>
__device__ __forceinline__ double kkt_apply(const Inst<T>& I, const double* p, double* q) {
  const int n = I.n, m = I.m;
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *dl = I.P(I.L.dl), *qd = I.P(I.L.qd);
  double *t = I.P(I.L.t), *wv = I.P(I.L.wv), *ya = I.P(I.L.ya), *yh = I.P(I.L.yh);
  if (m > 0) rowdots<false>(I.A, m, n, p, t);
  __syncthreads();
  double dot = 0.0;
  for (int i = threadIdx.x; i < m; i += kBB) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double pl = p[n + i], pu = p[n + m + i], dL = dl[i], dU = dl[m + i];
    const double ylo = (hl ? t[i] : 0.0) + dL * pl;
    const double yup = (hu ? -t[i] : 0.0) + dU * pu;
    q[n + i] = ylo;
    q[n + m + i] = yup;
    wv[i] = (hl ? 2.0 * t[i] / dL + pl : 0.0) - (hu ? -2.0 * t[i] / dU + pu : 0.0);
    dot += pl * ylo + pu * yup;
  }
  __syncthreads();
  if (m > 0) coldots<false>(I.A, m, n, wv, ya);
  __syncthreads();
  if (I.hk == 0) {
    rowdots<false>(I.H, n, n, p, yh);
    __syncthreads();
  } else {
    double *g = I.P(I.L.g), *gw = I.P(I.L.gw);
    coldots<false>(I.H, n, I.k, p, g);
    __syncthreads();
    for (int l = threadIdx.x; l < I.k; l += kBB) gw[l] = I.P(I.L.wd)[l] * g[l];
    __syncthreads();
    rowdots<false>(I.H, n, I.k, gw, yh);
    __syncthreads();
  }
  for (int j = threadIdx.x; j < n; j += kBB) {
    const double y = (m > 0 ? ya[j] : 0.0) + yh[j] + qd[j] * p[j];
    q[j] = y;
    dot += p[j] * y;
  }
  return wg_sum(dot);
}

// Jacobi PCG on eq. 9 into sol; returns iterations (negative: status code).
template <typename T>
__device__ __noinline__ int pcg(const BInst* bi, double* vec, double tol, int maxit,
                               int* converged_out) {
  const Inst<T> I(*bi, vec);
  const int N = I.n + 2 * I.m;
  double *x = I.P(I.L.sol), *r = I.P(I.L.r), *z = I.P(I.L.z), *p = I.P(I.L.p), *q = I.P(I.L.q);
  const double *rhs = I.P(I.L.rhs), *jd = I.P(I.L.jd);
  double rz = 0.0, rr = 0.0;
  for (int i = threadIdx.x; i < N; i += kBB) {
    const double ri = rhs[i], zi = ri / jd[i];
    x[i] = 0.0; r[i] = ri; z[i] = zi; p[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = wg_sum(rz);
  const double nb = sqrt(wg_sum(rr));
  *converged_out = 0;
  if (!(nb > 0.0)) {
    *converged_out = nb == 0.0;
    return nb == 0.0 ? 0 : QP_ERR_NUMERIC_CODE;
  }
  for (int k = 0; k < maxit; ++k) {
    const double pq = kkt_apply(I, p, q);
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz))
      return (isfinite(pq) && isfinite(rz)) ? QP_ERR_NOT_SPD_CODE : QP_ERR_NUMERIC_CODE;
    const double alpha = rz / pq;
    double rzn = 0.0, rn = 0.0;
    for (int i = threadIdx.x; i < N; i += kBB) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i], zi = ri / jd[i];
      r[i] = ri; z[i] = zi;
      rzn += ri * zi;
      rn += ri * ri;
    }
    rzn = wg_sum(rzn);
    rn = wg_sum(rn);
    if (sqrt(rn) <= tol * nb) {
      *converged_out = 1;
      return k + 1;
    }
    const double beta = rzn / rz;
    rz = rzn;
    for (int i = threadIdx.x; i < N; i += kBB) p[i] = z[i] + beta * p[i];
    __syncthreads();
  }
  return maxit;
}

// Recovery (eq. 7) and the ratio test (eq. 10): returns alpha_x, alpha_lam.
template <typename T>
__device__ __noinline__ void recover_ratio(const BInst* bi, double* vec, double gamma,
                                        double* alphas) {
  const Inst<T> I(*bi, vec);
  double ax, al;
  const int n = I.n, m = I.m;
  const double *lam = I.P(I.L.lam), *s = I.P(I.L.s), *res = I.P(I.L.res);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  double *dx = I.P(I.L.sol), *dlam = I.P(I.L.sol) + n, *ds = I.P(I.L.ds), *t = I.P(I.L.t);
  const int64_t olA = n, ouA = n + m, olx = n + 2 * m, oux = 2 * n + 2 * m, oc3 = 3 * n + 4 * m,
                oc4 = 4 * n + 4 * m;
  if (m > 0) rowdots<false>(I.A, m, n, dx, t);
  __syncthreads();
  double ms = INFINITY, ml = INFINITY;
  for (int i = threadIdx.x; i < m; i += kBB) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double dsl = hl ? t[i] + res[olA + i] : 0.0;
    const double dsu = hu ? -t[i] + res[ouA + i] : 0.0;
    ds[i] = dsl; ds[m + i] = dsu;
    const double dll = hl ? dlam[i] : 0.0, dlu = hu ? dlam[m + i] : 0.0;
    dlam[i] = dll; dlam[m + i] = dlu;
    if (hl && dsl < 0.0) ms = fmin(ms, -s[i] / dsl);
    if (hu && dsu < 0.0) ms = fmin(ms, -s[m + i] / dsu);
    if (hl && dll < 0.0) ml = fmin(ml, -lam[i] / dll);
    if (hu && dlu < 0.0) ml = fmin(ml, -lam[m + i] / dlu);
  }
  for (int j = threadIdx.x; j < n; j += kBB) {
    const bool hl = blo(lx[j]), hu = bhi(ux[j]);
    double dsl = 0.0, dsu = 0.0, dll = 0.0, dlu = 0.0;
    if (hl) {
      const double slx = s[2 * m + j], llx = lam[2 * m + j];
      dsl = dx[j] + res[olx + j];
      dll = -(res[oc3 + j] + llx * dsl) / slx;
      if (dsl < 0.0) ms = fmin(ms, -slx / dsl);
      if (dll < 0.0) ml = fmin(ml, -llx / dll);
    }
    if (hu) {
      const double sux = s[2 * m + n + j], lux = lam[2 * m + n + j];
      dsu = -dx[j] + res[oux + j];
      dlu = -(res[oc4 + j] + lux * dsu) / sux;
      if (dsu < 0.0) ms = fmin(ms, -sux / dsu);
      if (dlu < 0.0) ml = fmin(ml, -lux / dlu);
    }
    ds[2 * m + j] = dsl; ds[2 * m + n + j] = dsu;
    dlam[2 * m + j] = dll; dlam[2 * m + n + j] = dlu;
  }
  ms = wg_min(ms);
  ml = wg_min(ml);
  ax = fmin(1.0, gamma * ms);
  al = fmin(1.0, gamma * ml);
  alphas[0] = ax;
  alphas[1] = al;
}

template <typename T>
__device__ __forceinline__ void solve_one(const BArgs<T>& a, int id) {
  const Inst<T> I(a.inst[id], a.vec);
  const int n = I.n, m = I.m;
  const BOpts& o = a.o;
  double *x = I.P(I.L.x), *lam = I.P(I.L.lam), *s = I.P(I.L.s), *t = I.P(I.L.t);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  // diag(H)
  double* diagH = I.P(I.L.diagH);
  if (I.hk == 0) {
    for (int j = threadIdx.x; j < n; j += kBB) diagH[j] = static_cast<double>(I.H[static_cast<int64_t>(j) * n + j]);
  } else {
    rowdots<true>(I.H, n, I.k, I.P(I.L.wd), diagH);
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kBB) diagH[j] += I.P(I.L.h0)[j];
  }
  // starting point
  for (int j = threadIdx.x; j < n; j += kBB) {
    const bool hl = blo(lx[j]), hu = bhi(ux[j]);
    double xj = 0.0;
    if (hl && hu) xj = 0.5 * (lx[j] + ux[j]);
    else if (hl) xj = lx[j] + 1.0;
    else if (hu) xj = ux[j] - 1.0;
    x[j] = xj;
    s[2 * m + j] = hl ? xj - lx[j] : 0.0;
    s[2 * m + n + j] = hu ? ux[j] - xj : 0.0;
    lam[2 * m + j] = hl ? 1.0 : 0.0;
    lam[2 * m + n + j] = hu ? 1.0 : 0.0;
  }
  __syncthreads();
  if (m > 0) rowdots<false>(I.A, m, n, x, t);
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += kBB) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    s[i] = hl ? fmax(t[i] - lA[i], 1.0) : 0.0;
    s[m + i] = hu ? fmax(uA[i] - t[i], 1.0) : 0.0;
    lam[i] = hl ? 1.0 : 0.0;
    lam[m + i] = hu ? 1.0 : 0.0;
  }
  __syncthreads();
  double mu = o.mu0, nrm[4] = {0, 0, 0, 0};
  int it = 0, status = QP_IPM_MAX_ITER, hits = 0;
  int64_t total = 0;
  const BInst* bi = a.inst + id;
  for (it = 1; it <= o.max_iter; ++it) {
    residuals<T>(bi, a.vec, mu, nrm);
    newton_system<T>(bi, a.vec, mu);
    int conv = 0;
    const int pit = pcg<T>(bi, a.vec, o.cg_tol, o.cg_maxit, &conv);
    if (pit < 0) {
      status = pit;
      break;
    }
    total += pit;
    if (!conv) ++hits;
    double al2[2];
    recover_ratio<T>(bi, a.vec, o.gamma, al2);
    const double ax = al2[0], al = al2[1];
    const double *dx = I.P(I.L.sol), *dlam = I.P(I.L.sol) + n, *ds = I.P(I.L.ds);
    for (int j = threadIdx.x; j < n; j += kBB) x[j] += ax * dx[j];
    for (int q = threadIdx.x; q < 2 * m + 2 * n; q += kBB) {
      s[q] += ax * ds[q];      // absent sides carry zero steps
      lam[q] += al * dlam[q];
    }
    __syncthreads();
    residuals<T>(bi, a.vec, mu, nrm);
    if (!isfinite(nrm[0])) {
      status = QP_ERR_NUMERIC_CODE;
      break;
    }
    if (nrm[0] < mu) {
      if (mu < o.mu_tol) {
        status = QP_IPM_CONVERGED;
        break;
      }
      mu = mu / o.mu_div;
    }
  }
  // objective 1/2 x^T H x + c^T x
  double* yh = I.P(I.L.yh);
  hess_apply(I, x, yh);
  double ob = 0.0;
  const double* c = I.P(I.L.c);
  for (int j = threadIdx.x; j < n; j += kBB) ob += x[j] * (0.5 * yh[j] + c[j]);
  ob = wg_sum(ob);
  if (threadIdx.x == 0) {
    BResult r{};
    r.mu_final = mu; r.rnorm = nrm[0]; r.primal = nrm[1]; r.dual = nrm[2]; r.compl_ = nrm[3];
    r.objective = ob; r.status = status; r.iterations = it > o.max_iter ? o.max_iter : it;
    r.cg_hits = hits; r.total_cg = total;
    a.out[id] = r;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBB) void k_batch_ipm(BArgs<T> a) {
  __shared__ int slot;
  for (;;) {
    if (threadIdx.x == 0) slot = atomicAdd(a.next, 1);
    __syncthreads();
    // the slot is the same for the whole workgroup: make that visible to the
    // compiler so the instance's sizes and offsets live in scalar registers
    const int q = __builtin_amdgcn_readfirstlane(slot);
    __syncthreads();
    if (q >= a.count) break;
    solve_one(a, __builtin_amdgcn_readfirstlane(a.order[q]));
  }
}

// ---------------------------------------- allocation-free single dense solve
// The one instance's descriptor, queue counter, result and float64 block live
// in a fixed device array of the library, `scratch` (one per GPU, held until
// the process ends); H and A are read where the caller keeps them.
constexpr size_t kScratchBytes = size_t(16) << 20;
struct NaHead {
  BInst inst;
  int32_t order, next;
  BResult out;
  int32_t bad, pad;
};
constexpr size_t kNaHeadBytes = 256 * ((sizeof(NaHead) + 255) / 256);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Fills the instance's block from the caller's vectors (every entry, so a
// previous call's contents never leak in), checks the bounds, and writes the
// descriptor; an invalid problem leaves the queue empty, so the solve kernel
// exits at once.  One workgroup.
__global__ __launch_bounds__(kBB) void k_noalloc_setup(unsigned char* base, int n, int m, const double* H,
                                                       const double* A, const double* c, const double* lA,
                                                       const double* uA, const double* lx, const double* ux) {
  NaHead* hd = reinterpret_cast<NaHead*>(base);
  double* v = reinterpret_cast<double*>(base + kNaHeadBytes);
  const BLayout L(n, m, 0);
  for (int64_t i = threadIdx.x; i < L.total; i += kBB) v[i] = 0.0;
  __syncthreads();
  int bad = 0;
  for (int j = threadIdx.x; j < n; j += kBB) {
    const double l = lx ? lx[j] : -INFINITY, u = ux ? ux[j] : INFINITY;
    if (isnan(l) || isnan(u) || l == INFINITY || u == -INFINITY || (isfinite(l) && isfinite(u) && !(l < u)))
      bad = 1;
    v[L.c + j] = c[j];
    v[L.lx + j] = l;
    v[L.ux + j] = u;
  }
  for (int r = threadIdx.x; r < m; r += kBB) {
    const double l = lA[r], u = uA[r];
    if (isnan(l) || isnan(u) || l == INFINITY || u == -INFINITY || l > u) bad = 1;
    v[L.lA + r] = l;
    v[L.uA + r] = u;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    hd->inst.n = n;
    hd->inst.m = m;
    hd->inst.k = 0;
    hd->inst.hkind = 0;
    hd->inst.A = A;
    hd->inst.H = H;
    hd->inst.v_off = 0;
    hd->order = 0;
    hd->next = bad ? 1 : 0;
    hd->bad = bad;
    hd->out = BResult{};
  }
}

__global__ __launch_bounds__(kBB) void k_noalloc_out(const unsigned char* base, int n, int m, double* x,
                                                     double* lam, double* s) {
  const double* v = reinterpret_cast<const double*>(base + kNaHeadBytes);
  const BLayout L(n, m, 0);
  const int nl = 2 * m + 2 * n;
  for (int i = blockIdx.x * kBB + threadIdx.x; i < nl; i += gridDim.x * kBB) {
    if (x && i < n) x[i] = v[L.x + i];
    if (lam) lam[i] = v[L.lam + i];
    if (s) s[i] = v[L.s + i];
  }
}

}  // namespace qpk

using namespace qpk;

struct qp_batch_s {
  std::string err;
  hipStream_t st = nullptr;
  int count = 0;
  bool f32 = false;
  std::vector<BInst> inst;
  BInst* d_inst = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_next = nullptr;
  void* d_vals = nullptr;
  double* d_vec = nullptr;
  BResult* d_out = nullptr;
  std::vector<BResult> out;
  ~qp_batch_s() {
    for (void* p : {(void*)d_inst, (void*)d_order, (void*)d_next, d_vals, (void*)d_vec, (void*)d_out})
      if (p) (void)hipFree(p);
  }
};

#define BCHK(expr)                                                             \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      b->err = std::string(#expr) + ": " + hipGetErrorString(e_);              \
      return QP_ERR_HIP;                                                       \
    }                                                                          \
  } while (0)

static thread_local std::string g_batch_error;

extern "C" {

const char* qp_batch_last_error(qp_batch b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

static qp_status batch_create_impl(qp_batch b, const qp_desc* ds, int32_t count) {
  auto bad = [&](int i, const std::string& msg) {
    b->err = "instance " + std::to_string(i) + ": " + msg;
    return QP_ERR_ARG;
  };
  if (count < 1 || !ds) { b->err = "need count >= 1"; return QP_ERR_ARG; }
  const int prec = ds[0].precision;
  if (prec != QP_PREC_FP64 && prec != QP_PREC_FP32) {
    b->err = "batched solves store operators in float64 or float32";
    return QP_ERR_UNSUPPORTED;
  }
  b->f32 = prec == QP_PREC_FP32;
  const int vb = b->f32 ? 4 : 8;
  int64_t vals = 0, vecs = 0;
  b->inst.resize(count);
  std::vector<int64_t> a_off(count), h_off(count);   // element offsets in the value pool
  for (int i = 0; i < count; ++i) {
    const qp_desc& d = ds[i];
    if (d.precision != prec) return bad(i, "all instances need the same precision");
    if (d.n < 1 || d.m < 0) return bad(i, "need n >= 1, m >= 0");
    if (d.me != 0) { b->err = "batched solves take no equality rows"; return QP_ERR_UNSUPPORTED; }
    if (d.h_kind != QP_H_DENSE && d.h_kind != QP_H_LOWRANK) {
      b->err = "batched solves take a dense or low-rank H";
      return QP_ERR_UNSUPPORTED;
    }
    if (d.m > 0 && d.a_kind != QP_A_DENSE) {
      b->err = "batched solves take a dense A";
      return QP_ERR_UNSUPPORTED;
    }
    if (!d.c || (d.m > 0 && (!d.A || !d.lA || !d.uA))) return bad(i, "missing data");
    if (d.h_kind == QP_H_DENSE && !d.H) return bad(i, "missing H");
    if (d.h_kind == QP_H_LOWRANK && (d.k < 1 || !d.U || !d.wd || !d.h0)) return bad(i, "missing U, wd, h0");
    for (int64_t r = 0; r < d.m; ++r) {
      const double l = d.lA[r], u = d.uA[r];
      if (std::isnan(l) || std::isnan(u) || l == INFINITY || u == -INFINITY || l > u)
        return bad(i, "invalid row bounds");
    }
    for (int64_t j = 0; j < d.n; ++j) {
      const double l = d.lx ? d.lx[j] : -INFINITY, u = d.ux ? d.ux[j] : INFINITY;
      if (std::isnan(l) || std::isnan(u) || l == INFINITY || u == -INFINITY ||
          (std::isfinite(l) && std::isfinite(u) && !(l < u)))
        return bad(i, "invalid variable bounds");
    }
    BInst& I = b->inst[i];
    I.n = (int)d.n; I.m = (int)d.m; I.k = d.h_kind == QP_H_LOWRANK ? (int)d.k : 0;
    I.hkind = d.h_kind == QP_H_LOWRANK ? 1 : 0;
    a_off[i] = vals; vals += d.m * d.n;
    h_off[i] = vals; vals += I.hkind ? d.n * d.k : d.n * d.n;
    I.v_off = vecs; vecs += BLayout(I.n, I.m, I.k).total;
  }
  // host staging, then one upload each
  std::vector<double> hv(vecs, 0.0);
  std::vector<double> hval64;
  std::vector<float> hval32;
  if (b->f32) hval32.resize(vals); else hval64.resize(vals);
  auto put = [&](int64_t off, const double* src, int64_t cnt) {
    for (int64_t q = 0; q < cnt; ++q) {
      if (!std::isfinite(src[q])) return false;
      if (b->f32) hval32[off + q] = (float)src[q]; else hval64[off + q] = src[q];
    }
    return true;
  };
  for (int i = 0; i < count; ++i) {
    const qp_desc& d = ds[i];
    const BInst& I = b->inst[i];
    if (d.m > 0 && !put(a_off[i], d.A, d.m * d.n)) return bad(i, "A not finite");
    if (I.hkind ? !put(h_off[i], d.U, d.n * d.k) : !put(h_off[i], d.H, d.n * d.n)) return bad(i, "H not finite");
    const BLayout L(I.n, I.m, I.k);
    double* v = hv.data() + I.v_off;
    for (int64_t j = 0; j < d.n; ++j) {
      v[L.c + j] = d.c[j];
      v[L.h0 + j] = I.hkind ? d.h0[j] : 0.0;
      v[L.lx + j] = d.lx ? d.lx[j] : -INFINITY;
      v[L.ux + j] = d.ux ? d.ux[j] : INFINITY;
    }
    for (int l = 0; l < I.k; ++l) v[L.wd + l] = d.wd[l];
    for (int64_t r = 0; r < d.m; ++r) { v[L.lA + r] = d.lA[r]; v[L.uA + r] = d.uA[r]; }
  }
  // largest work first (longest-processing-time order for the queue)
  std::vector<int32_t> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto work = [&](int i) {
    const BInst& I = b->inst[i];
    return (double)I.m * I.n + (double)I.n * (I.hkind ? I.k : I.n);
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  b->count = count;
  BCHK(hipMalloc((void**)&b->d_inst, sizeof(BInst) * count));
  BCHK(hipMalloc((void**)&b->d_order, sizeof(int32_t) * count));
  BCHK(hipMalloc((void**)&b->d_next, sizeof(int32_t)));
  BCHK(hipMalloc(&b->d_vals, (size_t)std::max<int64_t>(vals, 1) * vb));
  BCHK(hipMalloc((void**)&b->d_vec, sizeof(double) * std::max<int64_t>(vecs, 1)));
  BCHK(hipMalloc((void**)&b->d_out, sizeof(BResult) * count));
  for (int i = 0; i < count; ++i) {
    b->inst[i].A = static_cast<const char*>(b->d_vals) + a_off[i] * vb;
    b->inst[i].H = static_cast<const char*>(b->d_vals) + h_off[i] * vb;
  }
  BCHK(hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, b->st));
  BCHK(hipMemcpyAsync(b->d_order, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, b->st));
  if (vals > 0)
    BCHK(hipMemcpyAsync(b->d_vals, b->f32 ? (const void*)hval32.data() : (const void*)hval64.data(),
                        (size_t)vals * vb, hipMemcpyHostToDevice, b->st));
  BCHK(hipMemcpyAsync(b->d_vec, hv.data(), sizeof(double) * vecs, hipMemcpyHostToDevice, b->st));
  BCHK(hipStreamSynchronize(b->st));
  b->out.resize(count);
  return QP_OK;
}

qp_status qp_batch_create(const qp_desc* ds, int32_t count, void* stream, qp_batch* out) {
  if (!out) return QP_ERR_ARG;
  *out = nullptr;
  qp_batch b = new (std::nothrow) qp_batch_s();
  if (!b) return QP_ERR_ALLOC;
  b->st = (hipStream_t)stream;
  qp_status s;
  try {
    s = batch_create_impl(b, ds, count);
  } catch (const std::bad_alloc&) {
    b->err = "host allocation failed";
    s = QP_ERR_ALLOC;
  }
  if (s != QP_OK) {
    g_batch_error = b->err;
    delete b;
    return s;
  }
  *out = b;
  return QP_OK;
}

void qp_batch_destroy(qp_batch b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->st);
  delete b;
}

qp_status ipm_solve_batch(qp_batch b, const ipm_options* o, int32_t workgroups, ipm_info* infos) {
  if (!b || !infos) return QP_ERR_ARG;
  ipm_options opt;
  qp_default_ipm_options(&opt);
  if (o) opt = *o;
  if (opt.warm_start) { b->err = "batched solves always start from the default point"; return QP_ERR_UNSUPPORTED; }
  if (opt.mu_rule != QP_MU_PAPER) { b->err = "batched solves run the paper's mu rule"; return QP_ERR_UNSUPPORTED; }
  BOpts bo{};
  bo.gamma = opt.gamma; bo.mu0 = opt.mu0; bo.mu_tol = opt.mu_tol; bo.mu_div = opt.mu_div;
  bo.max_iter = opt.max_iter;
  bo.cg_tol = opt.pcg.tol > 0 ? opt.pcg.tol : 1e-7;
  bo.cg_maxit = opt.pcg.maxit > 0 ? opt.pcg.maxit : 5000;
  if (!(bo.gamma > 0 && bo.gamma < 1) || !(bo.mu0 > 0) || !(bo.mu_div > 1) || bo.max_iter < 1) {
    b->err = "invalid ipm_options";
    return QP_ERR_ARG;
  }
  int grid = workgroups > 0 ? workgroups : 512;
  grid = std::min(grid, b->count);
  BCHK(hipMemsetAsync(b->d_next, 0, sizeof(int32_t), b->st));
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  BCHK(hipEventRecord(e0, b->st));
  if (b->f32) {
    BArgs<float> a{b->d_inst, b->d_order, b->count, b->d_next, b->d_vec, b->d_out, bo};
    k_batch_ipm<float><<<grid, kBB, 0, b->st>>>(a);
  } else {
    BArgs<double> a{b->d_inst, b->d_order, b->count, b->d_next, b->d_vec, b->d_out, bo};
    k_batch_ipm<double><<<grid, kBB, 0, b->st>>>(a);
  }
  BCHK(hipGetLastError());
  BCHK(hipEventRecord(e1, b->st));
  BCHK(hipMemcpyAsync(b->out.data(), b->d_out, sizeof(BResult) * b->count, hipMemcpyDeviceToHost, b->st));
  BCHK(hipStreamSynchronize(b->st));
  float ms = 0.f;
  BCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  qp_status worst = QP_OK;
  for (int i = 0; i < b->count; ++i) {
    const BResult& r = b->out[i];
    ipm_info& f = infos[i];
    std::memset(&f, 0, sizeof(f));
    f.result = r.status == QP_IPM_CONVERGED ? QP_IPM_CONVERGED : QP_IPM_MAX_ITER;
    f.iterations = r.iterations;
    f.total_cg_iters = r.total_cg;
    f.cg_maxiter_hits = r.cg_hits;
    f.mu_final = r.mu_final;
    f.rnorm = r.rnorm;
    f.primal = r.primal;
    f.dual = r.dual;
    f.compl_ = r.compl_;
    f.objective = r.objective;
    f.time_ms = ms;  // the one launch that solved the whole batch
    f.pcg_time_ms = 0.0;
    if (r.status == QP_ERR_NOT_SPD_CODE) worst = QP_ERR_NOT_SPD;
    else if (r.status == QP_ERR_NUMERIC_CODE && worst == QP_OK) worst = QP_ERR_NUMERIC;
  }
  if (worst != QP_OK) b->err = "at least one instance stopped on a numerical error (see its info)";
  return worst;
}

// Per-device address of `scratch`, looked up once per device with that
// device current (the array's name in host code is not a device address).
static std::mutex g_scratch_mu;
static void* g_scratch[64] = {};

static qp_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= 64) {
    g_batch_error = "device index out of range";
    return QP_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_batch_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return QP_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return QP_OK;
}

#define NCHK(expr)                                                             \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      g_batch_error = std::string(#expr) + ": " + hipGetErrorString(e_);       \
      return QP_ERR_HIP;                                                       \
    }                                                                          \
  } while (0)

qp_status ipm_solve_dense_noalloc(int64_t n, int64_t m, const double* H, const double* c,
                                  const double* A, const double* lA, const double* uA,
                                  const double* lx, const double* ux, const ipm_options* o,
                                  double* x, double* lam, double* s, ipm_info* info, void* stream) {
  if (n < 1 || m < 0 || n > INT32_MAX / 8 || m > INT32_MAX / 8 || !H || !c || !info ||
      (m > 0 && (!A || !lA || !uA))) {
    g_batch_error = "need n >= 1, m >= 0, H, c, info, and A, lA, uA when m > 0";
    return QP_ERR_ARG;
  }
  const size_t need = kNaHeadBytes + sizeof(double) * (size_t)BLayout(n, m, 0).total;
  if (need > kScratchBytes) {
    g_batch_error = "problem needs " + std::to_string(need) + " bytes of workspace; the allocation-free "
                    "solve has " + std::to_string(kScratchBytes) + " (it takes 29 n + 31 m float64 values)";
    return QP_ERR_ARG;
  }
  ipm_options opt;
  qp_default_ipm_options(&opt);
  if (o) opt = *o;
  if (opt.warm_start) {
    g_batch_error = "the allocation-free solve always starts from the default point";
    return QP_ERR_UNSUPPORTED;
  }
  if (opt.mu_rule != QP_MU_PAPER) {
    g_batch_error = "the allocation-free solve runs the paper's mu rule";
    return QP_ERR_UNSUPPORTED;
  }
  BOpts bo{};
  bo.gamma = opt.gamma; bo.mu0 = opt.mu0; bo.mu_tol = opt.mu_tol; bo.mu_div = opt.mu_div;
  bo.max_iter = opt.max_iter;
  bo.cg_tol = opt.pcg.tol > 0 ? opt.pcg.tol : 1e-7;
  bo.cg_maxit = opt.pcg.maxit > 0 ? opt.pcg.maxit : 5000;
  if (!(bo.gamma > 0 && bo.gamma < 1) || !(bo.mu0 > 0) || !(bo.mu_div > 1) || bo.max_iter < 1) {
    g_batch_error = "invalid ipm_options";
    return QP_ERR_ARG;
  }
  int dev = 0;
  NCHK(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  qp_status st = scratch_address(dev, &base);
  if (st != QP_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  NaHead* hd = reinterpret_cast<NaHead*>(base);
  k_noalloc_setup<<<1, kBB, 0, hs>>>(base, (int)n, (int)m, H, A, c, lA, uA, lx, ux);
  NCHK(hipGetLastError());
  BArgs<double> a{&hd->inst, &hd->order, 1, &hd->next, reinterpret_cast<double*>(base + kNaHeadBytes),
                  &hd->out, bo};
  k_batch_ipm<double><<<1, kBB, 0, hs>>>(a);
  NCHK(hipGetLastError());
  if (x || lam || s) {
    const int nl = (int)(2 * m + 2 * n);
    k_noalloc_out<<<std::min(256, (nl + kBB - 1) / kBB), kBB, 0, hs>>>(base, (int)n, (int)m, x, lam, s);
    NCHK(hipGetLastError());
  }
  BResult r{};
  int32_t bad = 0;
  NCHK(hipMemcpyAsync(&r, &hd->out, sizeof(BResult), hipMemcpyDeviceToHost, hs));
  NCHK(hipMemcpyAsync(&bad, &hd->bad, sizeof(int32_t), hipMemcpyDeviceToHost, hs));
  NCHK(hipStreamSynchronize(hs));
  if (bad) {
    g_batch_error = "invalid bounds (NaN, an infinite side on the wrong side, or lower above upper)";
    return QP_ERR_ARG;
  }
  std::memset(info, 0, sizeof(*info));
  info->result = r.status == QP_IPM_CONVERGED ? QP_IPM_CONVERGED : QP_IPM_MAX_ITER;
  info->iterations = r.iterations;
  info->total_cg_iters = r.total_cg;
  info->cg_maxiter_hits = r.cg_hits;
  info->mu_final = r.mu_final;
  info->rnorm = r.rnorm;
  info->primal = r.primal;
  info->dual = r.dual;
  info->compl_ = r.compl_;
  info->objective = r.objective;
  info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (r.status == QP_ERR_NOT_SPD_CODE) {
    g_batch_error = "PCG met a non-positive curvature p^T K p";
    return QP_ERR_NOT_SPD;
  }
  if (r.status == QP_ERR_NUMERIC_CODE) {
    g_batch_error = "NaN or Inf met in a reduction";
    return QP_ERR_NUMERIC;
  }
  return QP_OK;
}

qp_status qp_batch_get_solution(qp_batch b, int32_t i, double* x, double* lam, double* s) {
  if (!b || i < 0 || i >= b->count) return QP_ERR_ARG;
  const BInst& I = b->inst[i];
  const BLayout L(I.n, I.m, I.k);
  const int64_t nl = 2 * (int64_t)I.m + 2 * (int64_t)I.n;
  const double* base = b->d_vec + I.v_off;
  if (x) BCHK(hipMemcpyAsync(x, base + L.x, sizeof(double) * I.n, hipMemcpyDeviceToDevice, b->st));
  if (lam) BCHK(hipMemcpyAsync(lam, base + L.lam, sizeof(double) * nl, hipMemcpyDeviceToDevice, b->st));
  if (s) BCHK(hipMemcpyAsync(s, base + L.s, sizeof(double) * nl, hipMemcpyDeviceToDevice, b->st));
  BCHK(hipStreamSynchronize(b->st));
  return QP_OK;
}

}  // extern "C"
