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
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>
#include <type_traits>
#include <functional>

namespace qpk {

constexpr int kBB = 1024;            // threads per workgroup
constexpr int kBW = kBB / 64;        // waves per workgroup
constexpr int kTeamMax = 64;         // most workgroups in one team
constexpr int kRedSlots = 4;         // rotating slots of a team's reductions

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
  int32_t status, iterations, cg_hits, team;   // team: workgroups that solved it
  int64_t total_cg;
  int64_t t_start, t_end;                      // device wall clock around its solve
};

// A team's state in device memory: its barrier's arrival count (monotonic
// over the launch), the instance it is on, and each member's partials of the
// team's reductions, in rotating slots.
struct TeamSync {
  unsigned long long bar;
  int32_t cur, pad;
  double red[kRedSlots][kTeamMax][4];
};

// How a team launch is organised: workgroup w belongs to team team_of[w],
// whose members are workgroups first[t] .. first[t] + size[t] - 1; team t
// takes instances from queue queue[t], i.e. qorder[qstart[q] + i] for the
// i it draws from the counter qnext[q] (i < qcount[q]).  A wait at a team
// barrier gives up after spin_max polls and sets *abort; every team that
// meets a barrier after that leaves its instance and the launch (the results
// of that launch are invalid), so the grid drains instead of running on.
struct TeamPlan {
  const int32_t* team_of;
  const int32_t* first;
  const int32_t* size;
  const int32_t* queue;
  const int32_t* qstart;
  const int32_t* qcount;
  int32_t* qnext;
  const int32_t* qorder;
  TeamSync* sync;
  int32_t* abort;
  int32_t spin_max;
  int32_t nqueue;   // queues, by team size, largest first
  double* part;     // ld float64 per workgroup of the launch: column partial sums
  int32_t ld;
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
  TeamPlan plan;   // plan.team_of null: every workgroup a team of its own on `order`
};

__device__ __forceinline__ bool blo(double l) { return l > -INFINITY; }
__device__ __forceinline__ bool bhi(double u) { return u < INFINITY; }

// The workgroups solving one instance together.  Work is spread over the
// team's threads (tid, nthr), waves (wave, nwave) and column tiles; the
// team's phases are separated by team_sync.  A team of one is a workgroup:
// its barrier is __syncthreads and its reductions stay in LDS.
struct Team {
  int G, r;
  TeamSync* ts;
  int32_t* abort;
  int32_t spin_max;
  unsigned long long gen;   // barriers passed
  int slot;                 // next reduction slot
  int dead;                 // the launch was aborted: leave at once
  double* part;             // the team's column partial sums, member q at part + q * ld
  int ld;
  __device__ int tid() const { return r * kBB + static_cast<int>(threadIdx.x); }
  __device__ int nthr() const { return G * kBB; }
  __device__ int wave() const { return r * kBW + static_cast<int>(threadIdx.x >> 6); }
  __device__ int nwave() const { return G * kBW; }
};

// Team barrier: every member's writes so far are visible to every member
// after it.  Thread 0 of each member releases its workgroup's writes at
// device scope, counts its arrival and waits for the count of this barrier,
// then acquires; the workgroup's own barrier brackets it.  Every member
// then reads the launch's abort flag (set by a wait that gave up) into
// t.dead, so all of them leave at their next check.
__device__ __noinline__ void team_sync(Team& t) {
  __shared__ int aborted;
  __syncthreads();
  if (t.G == 1) return;
  ++t.gen;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(&t.ts->bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long target = t.gen * static_cast<unsigned long long>(t.G);
    int spin = 0;
    while (__hip_atomic_load(&t.ts->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(t.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++spin >= t.spin_max) {
        __hip_atomic_store(t.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    aborted = __hip_atomic_load(t.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  t.dead = aborted;
}

// Sums (MIN: minima) over the team of NV values per thread, the same bits on
// every thread of every member: each workgroup reduces by wave shuffles and
// then its waves in order; with several members their results are combined
// in rank order through the team's reduction slot.
template <int NV, bool MIN = false>
__device__ __forceinline__ void team_reduce(Team& t, double* v) {
  __shared__ double sh[4][kBW];
  __shared__ double res[4];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double w = __shfl_xor(v[k], o, 64);
      v[k] = MIN ? fmin(v[k], w) : v[k] + w;
    }
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double a = MIN ? INFINITY : 0.0;
#pragma unroll
    for (int i = 0; i < kBW; ++i) a = MIN ? fmin(a, sh[threadIdx.x][i]) : a + sh[threadIdx.x][i];
    res[threadIdx.x] = a;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = res[k];
  if (t.G == 1) {
    __syncthreads();
    return;
  }
  const int slot = t.slot;
  t.slot = (t.slot + 1) % kRedSlots;
  if (threadIdx.x < NV) t.ts->red[slot][t.r][threadIdx.x] = res[threadIdx.x];
  team_sync(t);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = MIN ? INFINITY : 0.0;
    for (int q = 0; q < t.G; ++q) a = MIN ? fmin(a, t.ts->red[slot][q][k]) : a + t.ts->red[slot][q][k];
    v[k] = a;
  }
}

__device__ __forceinline__ double team_sum(Team& t, double v) {
  team_reduce<1>(t, &v);
  return v;
}

// Loads in flight per lane in the operator loops below: each batch issues
// all of its loads before the first product, so a wave waits for one memory
// latency per batch instead of one per element.  What is left after the full
// batches goes in one more batch whose indexes are clamped to the last
// element (in bounds) and whose products past the end are zeroed, so short
// rows and columns do not fall back to one latency per element.  The
// products are added in the same order as one element at a time.
constexpr int kUnroll = 16;

// The operators and vectors live in device memory.  Addressing them as
// global memory (not flat) keeps the loads off the counter that LDS and
// scalar loads share, so a wait for either does not drain the operator
// loads in flight; the row and tile bases are made wave-uniform.
template <typename T>
using gmem = const __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* as_global(const T* p) {
  return (gmem<T>*)p;
}

// out[r] = sum_c M[r][c] * v[c] (SQ: M^2).  Each wave of the team takes
// kRowB rows at a time and walks them together, kColB columns per lane per
// batch: kRowB * kColB operator loads in flight per lane, one load of v for
// all kRowB rows, and a row shorter than a batch still shares its latency
// with the other rows.
constexpr int kRowB = 4;
template <bool SQ, typename T>
__device__ __noinline__ void rowdots(const Team& tm, const T* __restrict__ M, int R, int Cn,
                                        const double* __restrict__ v, double* __restrict__ out) {
  constexpr int kColB = sizeof(T) == 4 ? 4 : 2;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tm.wave());
  const int step = __builtin_amdgcn_readfirstlane(tm.nwave()) * kRowB;
  for (int r0 = wv * kRowB; r0 < R; r0 += step) {
    const int nr = min(kRowB, R - r0);
    double acc[kRowB];
#pragma unroll
    for (int q = 0; q < kRowB; ++q) acc[q] = 0.0;
    for (int c0 = 0; c0 < Cn; c0 += kColB * 64) {
      T a[kRowB][kColB];
      double vv[kColB];
      gmem<double>* vb = as_global(v + c0);
      if (__builtin_amdgcn_readfirstlane(nr == kRowB && c0 + kColB * 64 <= Cn)) {
#pragma unroll
        for (int u = 0; u < kColB; ++u) vv[u] = vb[lane + 64 * u];
#pragma unroll
        for (int q = 0; q < kRowB; ++q) {
          gmem<T>* rq = as_global(M + static_cast<int64_t>(r0 + q) * Cn + c0);
#pragma unroll
          for (int u = 0; u < kColB; ++u) a[q][u] = rq[lane + 64 * u];
        }
      } else {
        // the last batch of a row group: offsets clamped to the last column
        // and rows to the last row (all in bounds), values outside zeroed
        const int lim = Cn - 1 - c0;
        int off[kColB];
#pragma unroll
        for (int u = 0; u < kColB; ++u) off[u] = min(lane + 64 * u, lim);
#pragma unroll
        for (int u = 0; u < kColB; ++u) vv[u] = vb[off[u]];
#pragma unroll
        for (int q = 0; q < kRowB; ++q) {
          gmem<T>* rq = as_global(M + static_cast<int64_t>(r0 + min(q, nr - 1)) * Cn + c0);
#pragma unroll
          for (int u = 0; u < kColB; ++u) a[q][u] = rq[off[u]];
        }
#pragma unroll
        for (int u = 0; u < kColB; ++u) {
          const bool in = lane + 64 * u <= lim;
          vv[u] = in ? vv[u] : 0.0;
#pragma unroll
          for (int q = 0; q < kRowB; ++q) a[q][u] = (in && q < nr) ? a[q][u] : T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < kRowB; ++q)
#pragma unroll
        for (int u = 0; u < kColB; ++u) {
          const double d = static_cast<double>(a[q][u]);
          acc[q] += (SQ ? d * d : d) * vv[u];
        }
    }
#pragma unroll
    for (int q = 0; q < kRowB; ++q) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
      if (lane == 0 && q < nr) out[r0 + q] = acc[q];
    }
  }
}

// out[c] = sum_r M[r][c] * w[r] (SQ: M^2).  Wide operators (at least 768
// columns per member of the team): 1024-column tiles, one column per thread,
// each thread walking all rows in order, so a workgroup reads 4 KB of each
// of kUnroll consecutive rows per batch (close to a plain stream's rate).
// One workgroup on a narrow operator: 64-column tiles, sixteen row groups
// per tile, combined in LDS in group order.
constexpr int kTileW = 64, kTileRG = kBB / kTileW;
template <bool SQ, typename T>
__device__ __noinline__ void coldots_wide(const Team& tm, const T* __restrict__ M, int R, int Cn,
                                          const double* __restrict__ w, double* __restrict__ out) {
  gmem<double>* wg = as_global(w);
  for (int c0 = tm.r * kBB; c0 < Cn; c0 += kBB * tm.G) {
    const int c = c0 + static_cast<int>(threadIdx.x);
    const int off = min(static_cast<int>(threadIdx.x), Cn - 1 - c0);  // in bounds
    double acc = 0.0;
    for (int r = 0; r < R; r += kUnroll) {
      T a[kUnroll];
      if (r + kUnroll <= R) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) a[u] = as_global(M + static_cast<int64_t>(r + u) * Cn + c0)[off];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double d = static_cast<double>(a[u]);
          acc += (SQ ? d * d : d) * wg[r + u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          a[u] = as_global(M + static_cast<int64_t>(min(r + u, R - 1)) * Cn + c0)[off];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double d = r + u < R ? static_cast<double>(a[u]) : 0.0;
          const double ww = r + u < R ? wg[r + u] : 0.0;
          acc += (SQ ? d * d : d) * ww;
        }
      }
    }
    if (c < Cn) out[c] = acc;
  }
}

template <bool SQ, typename T>
__device__ __noinline__ void coldots_tiles(const Team& tm, const T* __restrict__ M, int R, int Cn,
                                           const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double red[kBB];
  gmem<double>* wg = as_global(w);
  const int cc = threadIdx.x & (kTileW - 1);
  const int rg = __builtin_amdgcn_readfirstlane(threadIdx.x / kTileW);  // one row group per wave
  for (int c0 = tm.r * kTileW; c0 < Cn; c0 += kTileW * tm.G) {
    const int c = c0 + cc;
    const int off = min(cc, Cn - 1 - c0);  // in bounds; the sum of c >= Cn is dropped
    double acc = 0.0;
    for (int r = rg; r < R; r += kTileRG * kUnroll) {
      T a[kUnroll];
      if (__builtin_amdgcn_readfirstlane(r + kTileRG * (kUnroll - 1) < R)) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          a[u] = as_global(M + static_cast<int64_t>(r + kTileRG * u) * Cn + c0)[off];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double d = static_cast<double>(a[u]);
          acc += (SQ ? d * d : d) * wg[r + kTileRG * u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          a[u] = as_global(M + static_cast<int64_t>(min(r + kTileRG * u, R - 1)) * Cn + c0)[off];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double d = r + kTileRG * u < R ? static_cast<double>(a[u]) : 0.0;
          const double ww = r + kTileRG * u < R ? wg[r + kTileRG * u] : 0.0;
          acc += (SQ ? d * d : d) * ww;
        }
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (rg == 0 && c < Cn) {
      double t = red[cc];
#pragma unroll
      for (int g = 1; g < kTileRG; ++g) t += red[g * kTileW + cc];
      out[c] = t;
    }
    __syncthreads();
  }
}

// A team too large for a wide tile each: every member sums its own slab of
// rows (R / G of them, in order) over all columns in 1,024-column tiles into
// its row of the team's partial sums; after a team barrier each member adds
// the G partials of its share of the columns in rank order.  The barrier at
// the end keeps the partials until every member has read them.
template <bool SQ, typename T>
__device__ __noinline__ void coldots_slabs(Team& tm, const T* __restrict__ M, int R, int Cn,
                                           const double* __restrict__ w, double* __restrict__ out) {
  gmem<double>* wg = as_global(w);
  const int r0 = static_cast<int>(static_cast<int64_t>(R) * tm.r / tm.G);
  const int r1 = static_cast<int>(static_cast<int64_t>(R) * (tm.r + 1) / tm.G);
  double* mine = tm.part + static_cast<int64_t>(tm.r) * tm.ld;
  for (int c0 = 0; c0 < Cn; c0 += kBB) {
    const int c = c0 + static_cast<int>(threadIdx.x);
    const int off = min(static_cast<int>(threadIdx.x), Cn - 1 - c0);  // in bounds
    double acc = 0.0;
    for (int r = r0; r < r1; r += kUnroll) {
      T a[kUnroll];
      if (r + kUnroll <= r1) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) a[u] = as_global(M + static_cast<int64_t>(r + u) * Cn + c0)[off];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double d = static_cast<double>(a[u]);
          acc += (SQ ? d * d : d) * wg[r + u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          a[u] = as_global(M + static_cast<int64_t>(min(r + u, r1 - 1)) * Cn + c0)[off];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double d = r + u < r1 ? static_cast<double>(a[u]) : 0.0;
          const double ww = r + u < r1 ? wg[r + u] : 0.0;
          acc += (SQ ? d * d : d) * ww;
        }
      }
    }
    if (c < Cn) mine[c] = acc;
  }
  team_sync(tm);
  for (int c = tm.tid(); c < Cn; c += tm.nthr()) {
    double t = 0.0;
    for (int q = 0; q < tm.G; ++q) t += tm.part[static_cast<int64_t>(q) * tm.ld + c];
    out[c] = t;
  }
  team_sync(tm);
}

// Wide operators: 1,024-column tiles, alternate members taking alternate
// tiles; a team larger than that sums row slabs (above); one workgroup on a
// narrow operator: 64-column tiles.
template <bool SQ, typename T>
__device__ __forceinline__ void coldots(Team& tm, const T* __restrict__ M, int R, int Cn,
                                        const double* __restrict__ w, double* __restrict__ out) {
  if (Cn >= 768 * tm.G) coldots_wide<SQ>(tm, M, R, Cn, w, out);
  else if (tm.G > 1) coldots_slabs<SQ>(tm, M, R, Cn, w, out);
  else coldots_tiles<SQ>(tm, M, R, Cn, w, out);
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

// y = H x into y (dense: row dots; low rank: h0 x + U (wd * (U^T x))).
template <typename T>
__device__ __forceinline__ void hess_apply(Team& tm, const Inst<T>& I, const double* x, double* y) {
  double* g = I.P(I.L.g);
  double* gw = I.P(I.L.gw);
  if (I.hk == 0) {
    rowdots<false>(tm, I.H, I.n, I.n, x, y);
    team_sync(tm);
    return;
  }
  coldots<false>(tm, I.H, I.n, I.k, x, g);
  team_sync(tm);
  for (int l = tm.tid(); l < I.k; l += tm.nthr()) gw[l] = I.P(I.L.wd)[l] * g[l];
  team_sync(tm);
  rowdots<false>(tm, I.H, I.n, I.k, gw, y);
  team_sync(tm);
  const double* h0 = I.P(I.L.h0);
  for (int j = tm.tid(); j < I.n; j += tm.nthr()) y[j] += h0[j] * x[j];
  team_sync(tm);
}

// Residual stack (eq. 3 with the bound rows) and its norms; returns
// {stacked, primal, dual, compl}.
template <typename T>
__device__ __noinline__ void residuals(Team& tm, const BInst* bi, double* vec, double mu,
                                       double* nrm) {
  const Inst<T> I(*bi, vec);
  const int n = I.n, m = I.m;
  const double *x = I.P(I.L.x), *lam = I.P(I.L.lam), *s = I.P(I.L.s);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  double *res = I.P(I.L.res), *t = I.P(I.L.t), *wv = I.P(I.L.wv), *ya = I.P(I.L.ya), *yh = I.P(I.L.yh);
  const int64_t oH = 0, olA = n, ouA = n + m, olx = n + 2 * m, oux = 2 * n + 2 * m,
                oc1 = 3 * n + 2 * m, oc2 = 3 * n + 3 * m, oc3 = 3 * n + 4 * m, oc4 = 4 * n + 4 * m;
  if (m > 0) rowdots<false>(tm, I.A, m, n, x, t);
  team_sync(tm);
  double v[3] = {0.0, 0.0, 0.0};   // primal, dual, compl
  for (int i = tm.tid(); i < m; i += tm.nthr()) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double ll = lam[i], lu = lam[m + i], sl = s[i], su = s[m + i];
    const double rl = hl ? t[i] - sl - lA[i] : 0.0;
    const double ru = hu ? -t[i] - su + uA[i] : 0.0;
    const double c1 = hl ? ll * sl - mu : 0.0;
    const double c2 = hu ? lu * su - mu : 0.0;
    res[olA + i] = rl; res[ouA + i] = ru; res[oc1 + i] = c1; res[oc2 + i] = c2;
    wv[i] = (hu ? lu : 0.0) - (hl ? ll : 0.0);
    v[0] += rl * rl + ru * ru;
    v[2] += c1 * c1 + c2 * c2;
  }
  team_sync(tm);
  if (m > 0) coldots<false>(tm, I.A, m, n, wv, ya);
  team_sync(tm);
  hess_apply(tm, I, x, yh);
  const double* c = I.P(I.L.c);
  for (int j = tm.tid(); j < n; j += tm.nthr()) {
    const bool hl = blo(lx[j]), hu = bhi(ux[j]);
    const double llx = hl ? lam[2 * m + j] : 0.0, lux = hu ? lam[2 * m + n + j] : 0.0;
    const double slx = s[2 * m + j], sux = s[2 * m + n + j];
    const double rH = yh[j] + c[j] + (m > 0 ? ya[j] : 0.0) - llx + lux;
    const double rlx = hl ? x[j] - slx - lx[j] : 0.0;
    const double rux = hu ? -x[j] - sux + ux[j] : 0.0;
    const double c3 = hl ? llx * slx - mu : 0.0;
    const double c4 = hu ? lux * sux - mu : 0.0;
    res[oH + j] = rH; res[olx + j] = rlx; res[oux + j] = rux; res[oc3 + j] = c3; res[oc4 + j] = c4;
    v[1] += rH * rH;
    v[0] += rlx * rlx + rux * rux;
    v[2] += c3 * c3 + c4 * c4;
  }
  team_reduce<3>(tm, v);
  nrm[0] = sqrt(v[0] + v[1] + v[2]);
  nrm[1] = sqrt(v[0]);
  nrm[2] = sqrt(v[1]);
  nrm[3] = sqrt(v[2]);
}

// D, the eq. 9 right-hand side, diag(K) and Q's diagonal (eqs. 8, 9).
template <typename T>
__device__ __noinline__ void newton_system(Team& tm, const BInst* bi, double* vec, double mu) {
  const Inst<T> I(*bi, vec);
  const int n = I.n, m = I.m;
  const double *lam = I.P(I.L.lam), *s = I.P(I.L.s), *res = I.P(I.L.res);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  double *rhs = I.P(I.L.rhs), *jd = I.P(I.L.jd), *dl = I.P(I.L.dl), *qd = I.P(I.L.qd);
  double *wv = I.P(I.L.wv), *jw = I.P(I.L.jw), *ya = I.P(I.L.ya), *yh = I.P(I.L.yh);
  const int64_t olA = n, ouA = n + m, olx = n + 2 * m, oux = 2 * n + 2 * m,
                oc1 = 3 * n + 2 * m, oc2 = 3 * n + 3 * m, oc3 = 3 * n + 4 * m, oc4 = 4 * n + 4 * m;
  for (int i = tm.tid(); i < m; i += tm.nthr()) {
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
  team_sync(tm);
  if (m > 0) {
    coldots<false>(tm, I.A, m, n, wv, ya);
    coldots<true>(tm, I.A, m, n, jw, yh);
  }
  team_sync(tm);
  const double *diagH = I.P(I.L.diagH), *h0 = I.P(I.L.h0);
  for (int j = tm.tid(); j < n; j += tm.nthr()) {
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
  team_sync(tm);
}

// q = K p (eq. 9, matrix-free); returns p . q.  The row products A p and, for
// a dense H, H p share the first phase (both only read p).
template <typename T>
__device__ __forceinline__ double kkt_apply(Team& tm, const Inst<T>& I, const double* p, double* q) {
  const int n = I.n, m = I.m;
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *dl = I.P(I.L.dl), *qd = I.P(I.L.qd);
  double *t = I.P(I.L.t), *wv = I.P(I.L.wv), *ya = I.P(I.L.ya), *yh = I.P(I.L.yh);
  if (m > 0) rowdots<false>(tm, I.A, m, n, p, t);
  if (I.hk == 0) rowdots<false>(tm, I.H, n, n, p, yh);
  team_sync(tm);
  double dot = 0.0;
  for (int i = tm.tid(); i < m; i += tm.nthr()) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double pl = p[n + i], pu = p[n + m + i], dL = dl[i], dU = dl[m + i];
    const double ylo = (hl ? t[i] : 0.0) + dL * pl;
    const double yup = (hu ? -t[i] : 0.0) + dU * pu;
    q[n + i] = ylo;
    q[n + m + i] = yup;
    wv[i] = (hl ? 2.0 * t[i] / dL + pl : 0.0) - (hu ? -2.0 * t[i] / dU + pu : 0.0);
    dot += pl * ylo + pu * yup;
  }
  team_sync(tm);
  if (m > 0) coldots<false>(tm, I.A, m, n, wv, ya);
  if (I.hk != 0) {
    double *g = I.P(I.L.g), *gw = I.P(I.L.gw);
    team_sync(tm);
    coldots<false>(tm, I.H, n, I.k, p, g);
    team_sync(tm);
    for (int l = tm.tid(); l < I.k; l += tm.nthr()) gw[l] = I.P(I.L.wd)[l] * g[l];
    team_sync(tm);
    rowdots<false>(tm, I.H, n, I.k, gw, yh);
  }
  team_sync(tm);
  for (int j = tm.tid(); j < n; j += tm.nthr()) {
    const double y = (m > 0 ? ya[j] : 0.0) + yh[j] + qd[j] * p[j];
    q[j] = y;
    dot += p[j] * y;
  }
  return team_sum(tm, dot);
}

// Jacobi PCG on eq. 9 into sol; returns iterations (negative: status code).
template <typename T>
__device__ __noinline__ int pcg(Team& tm, const BInst* bi, double* vec, double tol, int maxit,
                               int* converged_out) {
  const Inst<T> I(*bi, vec);
  const int N = I.n + 2 * I.m;
  double *x = I.P(I.L.sol), *r = I.P(I.L.r), *z = I.P(I.L.z), *p = I.P(I.L.p), *q = I.P(I.L.q);
  const double *rhs = I.P(I.L.rhs), *jd = I.P(I.L.jd);
  double v[2] = {0.0, 0.0};   // r.z, r.r
  for (int i = tm.tid(); i < N; i += tm.nthr()) {
    const double ri = rhs[i], zi = ri / jd[i];
    x[i] = 0.0; r[i] = ri; z[i] = zi; p[i] = zi;
    v[0] += ri * zi;
    v[1] += ri * ri;
  }
  team_reduce<2>(tm, v);
  double rz = v[0];
  const double nb = sqrt(v[1]);
  *converged_out = 0;
  if (!(nb > 0.0)) {
    *converged_out = nb == 0.0;
    return nb == 0.0 ? 0 : QP_ERR_NUMERIC_CODE;
  }
  for (int k = 0; k < maxit; ++k) {
    if (tm.dead) return QP_ERR_NUMERIC_CODE;
    const double pq = kkt_apply(tm, I, p, q);
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz))
      return (isfinite(pq) && isfinite(rz)) ? QP_ERR_NOT_SPD_CODE : QP_ERR_NUMERIC_CODE;
    const double alpha = rz / pq;
    double w[2] = {0.0, 0.0};   // r.z, r.r of the new residual
    for (int i = tm.tid(); i < N; i += tm.nthr()) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i], zi = ri / jd[i];
      r[i] = ri; z[i] = zi;
      w[0] += ri * zi;
      w[1] += ri * ri;
    }
    team_reduce<2>(tm, w);
    if (sqrt(w[1]) <= tol * nb) {
      *converged_out = 1;
      return k + 1;
    }
    const double beta = w[0] / rz;
    rz = w[0];
    for (int i = tm.tid(); i < N; i += tm.nthr()) p[i] = z[i] + beta * p[i];
    team_sync(tm);
  }
  return maxit;
}

// Recovery (eq. 7) and the ratio test (eq. 10): returns alpha_x, alpha_lam.
template <typename T>
__device__ __noinline__ void recover_ratio(Team& tm, const BInst* bi, double* vec, double gamma,
                                           double* alphas) {
  const Inst<T> I(*bi, vec);
  const int n = I.n, m = I.m;
  const double *lam = I.P(I.L.lam), *s = I.P(I.L.s), *res = I.P(I.L.res);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  double *dx = I.P(I.L.sol), *dlam = I.P(I.L.sol) + n, *ds = I.P(I.L.ds), *t = I.P(I.L.t);
  const int64_t olA = n, ouA = n + m, olx = n + 2 * m, oux = 2 * n + 2 * m, oc3 = 3 * n + 4 * m,
                oc4 = 4 * n + 4 * m;
  if (m > 0) rowdots<false>(tm, I.A, m, n, dx, t);
  team_sync(tm);
  double mn[2] = {INFINITY, INFINITY};   // slacks, multipliers
  for (int i = tm.tid(); i < m; i += tm.nthr()) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    const double dsl = hl ? t[i] + res[olA + i] : 0.0;
    const double dsu = hu ? -t[i] + res[ouA + i] : 0.0;
    ds[i] = dsl; ds[m + i] = dsu;
    const double dll = hl ? dlam[i] : 0.0, dlu = hu ? dlam[m + i] : 0.0;
    dlam[i] = dll; dlam[m + i] = dlu;
    if (hl && dsl < 0.0) mn[0] = fmin(mn[0], -s[i] / dsl);
    if (hu && dsu < 0.0) mn[0] = fmin(mn[0], -s[m + i] / dsu);
    if (hl && dll < 0.0) mn[1] = fmin(mn[1], -lam[i] / dll);
    if (hu && dlu < 0.0) mn[1] = fmin(mn[1], -lam[m + i] / dlu);
  }
  for (int j = tm.tid(); j < n; j += tm.nthr()) {
    const bool hl = blo(lx[j]), hu = bhi(ux[j]);
    double dsl = 0.0, dsu = 0.0, dll = 0.0, dlu = 0.0;
    if (hl) {
      const double slx = s[2 * m + j], llx = lam[2 * m + j];
      dsl = dx[j] + res[olx + j];
      dll = -(res[oc3 + j] + llx * dsl) / slx;
      if (dsl < 0.0) mn[0] = fmin(mn[0], -slx / dsl);
      if (dll < 0.0) mn[1] = fmin(mn[1], -llx / dll);
    }
    if (hu) {
      const double sux = s[2 * m + n + j], lux = lam[2 * m + n + j];
      dsu = -dx[j] + res[oux + j];
      dlu = -(res[oc4 + j] + lux * dsu) / sux;
      if (dsu < 0.0) mn[0] = fmin(mn[0], -sux / dsu);
      if (dlu < 0.0) mn[1] = fmin(mn[1], -lux / dlu);
    }
    ds[2 * m + j] = dsl; ds[2 * m + n + j] = dsu;
    dlam[2 * m + j] = dll; dlam[2 * m + n + j] = dlu;
  }
  team_reduce<2, true>(tm, mn);
  alphas[0] = fmin(1.0, gamma * mn[0]);
  alphas[1] = fmin(1.0, gamma * mn[1]);
}

template <typename T>
__device__ __forceinline__ void solve_one(Team& tm, const BArgs<T>& a, int id) {
  const int64_t t_start = wall_clock64();
  const Inst<T> I(a.inst[id], a.vec);
  const int n = I.n, m = I.m;
  const BOpts& o = a.o;
  double *x = I.P(I.L.x), *lam = I.P(I.L.lam), *s = I.P(I.L.s), *t = I.P(I.L.t);
  const double *lA = I.P(I.L.lA), *uA = I.P(I.L.uA), *lx = I.P(I.L.lx), *ux = I.P(I.L.ux);
  // diag(H)
  double* diagH = I.P(I.L.diagH);
  if (I.hk == 0) {
    for (int j = tm.tid(); j < n; j += tm.nthr())
      diagH[j] = static_cast<double>(I.H[static_cast<int64_t>(j) * n + j]);
  } else {
    rowdots<true>(tm, I.H, n, I.k, I.P(I.L.wd), diagH);
    team_sync(tm);
    for (int j = tm.tid(); j < n; j += tm.nthr()) diagH[j] += I.P(I.L.h0)[j];
  }
  // starting point
  for (int j = tm.tid(); j < n; j += tm.nthr()) {
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
  team_sync(tm);
  if (m > 0) rowdots<false>(tm, I.A, m, n, x, t);
  team_sync(tm);
  for (int i = tm.tid(); i < m; i += tm.nthr()) {
    const bool hl = blo(lA[i]), hu = bhi(uA[i]);
    s[i] = hl ? fmax(t[i] - lA[i], 1.0) : 0.0;
    s[m + i] = hu ? fmax(uA[i] - t[i], 1.0) : 0.0;
    lam[i] = hl ? 1.0 : 0.0;
    lam[m + i] = hu ? 1.0 : 0.0;
  }
  team_sync(tm);
  double mu = o.mu0, nrm[4] = {0, 0, 0, 0};
  int it = 0, status = QP_IPM_MAX_ITER, hits = 0;
  int64_t total = 0;
  const BInst* bi = a.inst + id;
  for (it = 1; it <= o.max_iter && !tm.dead; ++it) {
    residuals<T>(tm, bi, a.vec, mu, nrm);
    newton_system<T>(tm, bi, a.vec, mu);
    int conv = 0;
    const int pit = pcg<T>(tm, bi, a.vec, o.cg_tol, o.cg_maxit, &conv);
    if (pit < 0) {
      status = pit;
      break;
    }
    total += pit;
    if (!conv) ++hits;
    double al2[2];
    recover_ratio<T>(tm, bi, a.vec, o.gamma, al2);
    const double ax = al2[0], al = al2[1];
    const double *dx = I.P(I.L.sol), *dlam = I.P(I.L.sol) + n, *ds = I.P(I.L.ds);
    for (int j = tm.tid(); j < n; j += tm.nthr()) x[j] += ax * dx[j];
    for (int q = tm.tid(); q < 2 * m + 2 * n; q += tm.nthr()) {
      s[q] += ax * ds[q];      // absent sides carry zero steps
      lam[q] += al * dlam[q];
    }
    team_sync(tm);
    residuals<T>(tm, bi, a.vec, mu, nrm);
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
  hess_apply(tm, I, x, yh);
  double ob = 0.0;
  const double* c = I.P(I.L.c);
  for (int j = tm.tid(); j < n; j += tm.nthr()) ob += x[j] * (0.5 * yh[j] + c[j]);
  ob = team_sum(tm, ob);
  if (tm.r == 0 && threadIdx.x == 0) {
    BResult r{};
    r.mu_final = mu; r.rnorm = nrm[0]; r.primal = nrm[1]; r.dual = nrm[2]; r.compl_ = nrm[3];
    r.objective = ob; r.status = status; r.iterations = it > o.max_iter ? o.max_iter : it;
    r.cg_hits = hits; r.total_cg = total; r.team = tm.G;
    r.t_start = t_start; r.t_end = wall_clock64();
    a.out[id] = r;
  }
  team_sync(tm);
}

// Every workgroup belongs to a team (of one without a plan); a team draws
// instances from its queue until the queue is empty, then helps the queues
// of smaller team sizes (smaller instances) in turn.  The team's first member
// draws and passes the index to the others through the team's state.
template <typename T>
__global__ __launch_bounds__(kBB) void k_batch_ipm(BArgs<T> a) {
  __shared__ int slot;
  Team tm;
  tm.G = 1; tm.r = 0; tm.ts = nullptr; tm.abort = nullptr; tm.spin_max = 0; tm.dead = 0;
  tm.part = nullptr; tm.ld = 0;
  int home = 0, nq = 1;
  if (a.plan.team_of) {
    const int t = a.plan.team_of[blockIdx.x];
    tm.G = a.plan.size[t];
    tm.r = static_cast<int>(blockIdx.x) - a.plan.first[t];
    tm.ts = a.plan.sync + t;
    tm.abort = a.plan.abort;
    tm.spin_max = a.plan.spin_max;
    home = a.plan.queue[t];
    nq = a.plan.nqueue;
    tm.part = a.plan.part + static_cast<int64_t>(a.plan.first[t]) * a.plan.ld;
    tm.ld = a.plan.ld;
  }
  tm.gen = 0;
  tm.slot = 0;
  for (int qq = home; qq < nq && !tm.dead; ++qq) {
    const int32_t* order = a.plan.team_of ? a.plan.qorder + a.plan.qstart[qq] : a.order;
    const int32_t count = a.plan.team_of ? a.plan.qcount[qq] : a.count;
    int32_t* next = a.plan.team_of ? a.plan.qnext + qq : a.next;
    for (;;) {
      if (tm.r == 0 && threadIdx.x == 0) {
        slot = atomicAdd(next, 1);
        if (tm.G > 1) tm.ts->cur = slot;
      }
      team_sync(tm);
      if (tm.r != 0 && threadIdx.x == 0) slot = tm.ts->cur;
      __syncthreads();
      // the slot is the same for the whole workgroup: make that visible to the
      // compiler so the instance's sizes and offsets live in scalar registers
      const int q = __builtin_amdgcn_readfirstlane(slot);
      __syncthreads();
      if (q >= count || tm.dead) break;
      solve_one(tm, a, __builtin_amdgcn_readfirstlane(order[q]));
    }
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
  // team launches: the team size of each instance (all 1: one workgroup each)
  std::vector<int32_t> team;
  // the autotuner's estimate of each instance's PCG iteration on its team
  // (us; empty when the sizes came from qp_batch_set_teams)
  std::vector<double> t_est;
  int32_t* d_plan = nullptr;      // team_of | first | size | queue | qstart | qcount | qnext | qorder | abort
  int64_t plan_cap = 0;           // int32 entries of d_plan
  TeamSync* d_sync = nullptr;
  int sync_cap = 0;
  double* d_part = nullptr;       // column partial sums of team members: part_ld per workgroup
  int64_t part_cap = 0;           // float64 entries of d_part
  int32_t part_ld = 1;            // the largest column count of any operator (n or k)
  int last_grid = 0, last_teams = 0;
  bool have_out = false;          // out holds a completed launch's results
  ~qp_batch_s() {
    for (void* p : {(void*)d_inst, (void*)d_order, (void*)d_next, d_vals, (void*)d_vec, (void*)d_out,
                    (void*)d_plan, (void*)d_sync, (void*)d_part})
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
    b->part_ld = std::max(b->part_ld, std::max(I.n, I.k));
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
  b->team.assign(count, 1);
  return QP_OK;
}

// Work of one PCG iteration of an instance (operator entries read).
static double inst_work(const BInst& I) {
  return 2.0 * I.m * (double)I.n + (double)I.n * (I.hkind ? 2.0 * I.k : (double)I.n);
}

// Workgroups of the batch kernel that fit on the device at once.
static qp_status coresident(qp_batch b, int* out) {
  int dev = 0, cus = 0, per = 0;
  BCHK(hipGetDevice(&dev));
  BCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (b->f32) BCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_ipm<float>, kBB, 0));
  else BCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_ipm<double>, kBB, 0));
  *out = std::max(1, cus * per);
  return QP_OK;
}

// Plans a team launch on at most `cap` workgroups: the instances of each team
// size form a queue (largest work first); each size gets workgroups in
// proportion to its instances' work, as whole teams (at least one).
// Polls of a team barrier before it gives up (about 1 us each: a member
// lags its team by at most one phase of one instance, milliseconds).
// QPK_BATCH_SPIN overrides it (at least 1), so tests can force the give-up.
static int32_t team_spin_limit() {
  int32_t lim = 1 << 23;
  if (const char* e = std::getenv("QPK_BATCH_SPIN")) lim = std::max(1, std::atoi(e));
  return lim;
}

// Room for `wgs` workgroups' column partial sums (grown, never shrunk).
static qp_status ensure_part(qp_batch b, int wgs) {
  const int64_t need = static_cast<int64_t>(wgs) * b->part_ld;
  if (need > b->part_cap) {
    if (b->d_part) (void)hipFree(b->d_part);
    b->d_part = nullptr;
    b->part_cap = 0;
    BCHK(hipMalloc((void**)&b->d_part, sizeof(double) * need));
    b->part_cap = need;
  }
  return QP_OK;
}

static qp_status build_plan(qp_batch b, int cap, TeamPlan* plan, int* grid) {
  std::vector<int> sizes;
  for (int g : b->team) if (std::find(sizes.begin(), sizes.end(), g) == sizes.end()) sizes.push_back(g);
  std::sort(sizes.begin(), sizes.end(), std::greater<int>());
  const int nq = (int)sizes.size();
  std::vector<double> qwork(nq, 0.0);
  std::vector<std::vector<int32_t>> qinst(nq);
  // an instance's weight: the autotuner's estimate of its iteration on its
  // team (workgroup time = that times the team), else its operator work
  const bool est = b->t_est.size() == static_cast<size_t>(b->count);
  auto weight = [&](int i) { return est ? b->t_est[i] : inst_work(b->inst[i]); };
  std::vector<int32_t> order(b->count);
  for (int i = 0; i < b->count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return weight(x) > weight(y); });
  for (int i : order) {
    const int q = (int)(std::find(sizes.begin(), sizes.end(), b->team[i]) - sizes.begin());
    qinst[q].push_back(i);
    qwork[q] += est ? b->t_est[i] * sizes[q] : inst_work(b->inst[i]);
  }
  double tot = 0.0;
  for (double w : qwork) tot += w;
  // teams per queue: at least one, at most one per instance, within cap
  std::vector<int> nteams(nq, 1);
  int used = 0;
  for (int q = 0; q < nq; ++q) used += sizes[q];
  if (used > cap) {
    b->err = "team sizes need " + std::to_string(used) + " workgroups at once; " + std::to_string(cap) +
             " fit on the device";
    return QP_ERR_ARG;
  }
  for (int q = 0; q < nq; ++q) {
    const int want = (int)((double)cap * qwork[q] / std::max(tot, 1e-300) / sizes[q]);
    nteams[q] = std::max(1, std::min<int>((int)qinst[q].size(), want));
  }
  auto total_wg = [&]() {
    int t = 0;
    for (int q = 0; q < nq; ++q) t += nteams[q] * sizes[q];
    return t;
  };
  while (total_wg() > cap) {   // trim the queue with the most workgroups per unit of work
    int worst = -1;
    double ratio = -1.0;
    for (int q = 0; q < nq; ++q)
      if (nteams[q] > 1) {
        const double r = nteams[q] * sizes[q] / std::max(qwork[q], 1e-300);
        if (r > ratio) { ratio = r; worst = q; }
      }
    if (worst < 0) break;
    --nteams[worst];
  }
  if (est) {
    // with estimates: simulate each queue (its teams taking its instances in
    // order, each as soon as it is free) and move workgroups from the queue
    // that finishes first to the one that finishes last while that helps
    auto finish = [&](int q, int nt) {
      std::vector<double> free_at(std::max(nt, 1), 0.0);
      for (int i : qinst[q]) {
        auto it = std::min_element(free_at.begin(), free_at.end());
        *it += b->t_est[i];
      }
      return *std::max_element(free_at.begin(), free_at.end());
    };
    for (int step = 0; step < 4 * cap; ++step) {
      int qmax = 0, qmin = -1;
      std::vector<double> fin(nq);
      for (int q = 0; q < nq; ++q) {
        fin[q] = finish(q, nteams[q]);
        if (fin[q] > fin[qmax]) qmax = q;
      }
      if (nteams[qmax] >= (int)qinst[qmax].size()) break;   // one team per instance already
      const double gain = finish(qmax, nteams[qmax] + 1);
      if (total_wg() + sizes[qmax] <= cap) {
        ++nteams[qmax];
        continue;
      }
      // free sizes[qmax] workgroups from the queue that would finish first
      // without them
      double best = INFINITY;
      for (int q = 0; q < nq; ++q) {
        if (q == qmax) continue;
        const int drop = (sizes[qmax] + sizes[q] - 1) / sizes[q];
        if (nteams[q] - drop < 1) continue;
        const double f = finish(q, nteams[q] - drop);
        if (f < best) { best = f; qmin = q; }
      }
      if (qmin < 0 || !(std::max(best, gain) < fin[qmax])) break;
      nteams[qmin] -= (sizes[qmax] + sizes[qmin] - 1) / sizes[qmin];
      ++nteams[qmax];
    }
  }
  int teams = 0;
  for (int q = 0; q < nq; ++q) teams += nteams[q];
  const int W = total_wg();
  // host arrays, one upload
  std::vector<int32_t> team_of(W), first(teams), size(teams), queue(teams), qstart(nq), qcount(nq),
      qnext(nq, 0), qorder;
  int t = 0, w = 0;
  for (int q = 0; q < nq; ++q) {
    qstart[q] = (int32_t)qorder.size();
    qcount[q] = (int32_t)qinst[q].size();
    qorder.insert(qorder.end(), qinst[q].begin(), qinst[q].end());
    for (int k = 0; k < nteams[q]; ++k, ++t) {
      first[t] = w;
      size[t] = sizes[q];
      queue[t] = q;
      for (int r = 0; r < sizes[q]; ++r) team_of[w++] = t;
    }
  }
  std::vector<int32_t> blob;
  auto put = [&](const std::vector<int32_t>& v) {
    const int64_t off = (int64_t)blob.size();
    blob.insert(blob.end(), v.begin(), v.end());
    return off;
  };
  const int64_t o_team = put(team_of), o_first = put(first), o_size = put(size), o_queue = put(queue),
                o_qstart = put(qstart), o_qcount = put(qcount), o_qnext = put(qnext),
                o_qorder = put(qorder), o_abort = put({0});
  if ((int64_t)blob.size() > b->plan_cap) {
    if (b->d_plan) (void)hipFree(b->d_plan);
    b->d_plan = nullptr;
    b->plan_cap = 0;
    BCHK(hipMalloc((void**)&b->d_plan, sizeof(int32_t) * blob.size()));
    b->plan_cap = (int64_t)blob.size();
  }
  if (teams > b->sync_cap) {
    if (b->d_sync) (void)hipFree(b->d_sync);
    b->d_sync = nullptr;
    b->sync_cap = 0;
    BCHK(hipMalloc((void**)&b->d_sync, sizeof(TeamSync) * teams));
    b->sync_cap = teams;
  }
  BCHK(hipMemcpyAsync(b->d_plan, blob.data(), sizeof(int32_t) * blob.size(), hipMemcpyHostToDevice, b->st));
  BCHK(hipMemsetAsync(b->d_sync, 0, sizeof(TeamSync) * teams, b->st));
  int32_t* P = b->d_plan;
  plan->team_of = P + o_team; plan->first = P + o_first; plan->size = P + o_size;
  plan->queue = P + o_queue; plan->qstart = P + o_qstart; plan->qcount = P + o_qcount;
  plan->qnext = P + o_qnext; plan->qorder = P + o_qorder; plan->sync = b->d_sync;
  plan->abort = P + o_abort;
  plan->spin_max = team_spin_limit();
  plan->nqueue = nq;
  qp_status ps = ensure_part(b, W);
  if (ps != QP_OK) return ps;
  plan->part = b->d_part;
  plan->ld = b->part_ld;
  *grid = W;
  b->last_grid = W;
  b->last_teams = teams;
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
  const bool teams = std::any_of(b->team.begin(), b->team.end(), [](int g) { return g > 1; });
  TeamPlan plan{};
  int grid = workgroups > 0 ? workgroups : 512;
  if (teams) {
    // every member of a team must be resident while it waits for the others:
    // a cooperative launch within the device's co-resident workgroups
    int cap = 0;
    qp_status cs = coresident(b, &cap);
    if (cs != QP_OK) return cs;
    if (workgroups > 0) cap = std::min(cap, workgroups);
    cs = build_plan(b, cap, &plan, &grid);
    if (cs != QP_OK) return cs;
  } else {
    grid = std::min(grid, b->count);
    b->last_grid = grid;
    b->last_teams = grid;
  }
  BCHK(hipMemsetAsync(b->d_next, 0, sizeof(int32_t), b->st));
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  BCHK(hipEventRecord(e0, b->st));
  auto go = [&](auto* tag) -> hipError_t {
    using T = std::remove_pointer_t<decltype(tag)>;
    BArgs<T> a{b->d_inst, b->d_order, b->count, b->d_next, b->d_vec, b->d_out, bo, plan};
    if (!teams) {
      k_batch_ipm<T><<<grid, kBB, 0, b->st>>>(a);
      return hipGetLastError();
    }
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch_ipm<T>), dim3(grid),
                                      dim3(kBB), args, 0, b->st);
  };
  BCHK(b->f32 ? go((float*)nullptr) : go((double*)nullptr));
  BCHK(hipEventRecord(e1, b->st));
  b->have_out = false;
  BCHK(hipMemcpyAsync(b->out.data(), b->d_out, sizeof(BResult) * b->count, hipMemcpyDeviceToHost, b->st));
  BCHK(hipStreamSynchronize(b->st));
  b->have_out = true;
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
  if (teams) {
    int32_t ab = 0;
    BCHK(hipMemcpy(&ab, plan.abort, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (ab) {
      b->err = "a team barrier wait gave up (members not resident together): results invalid";
      return QP_ERR_HIP;
    }
  }
  if (worst != QP_OK) b->err = "at least one instance stopped on a numerical error (see its info)";
  return worst;
}

// ------------------------------------------------------------ autotuner
// Team sizes chosen from measured times.  Instances fall into classes by
// operator precision, H kind and the binary order of magnitude of the bytes
// one PCG iteration reads (2mn + n^2 or 2mn + 2nk values).  For each class
// its largest instance is timed alone with teams of 1, 2, 4, ... workgroups:
// one IPM iteration capped at kProbeIters PCG iterations, the time per PCG
// iteration taken from events around the launch.  The measurements are kept
// in a text table (one line per measurement: device architecture, precision,
// H kind, class, team size, microseconds per PCG iteration) that later calls
// read instead of timing again.  An instance's iteration time in the batch
// is the larger of its class's measured time (scaled by its share of the
// representative's work) and its operator bytes over its team's share of the
// chip's bandwidth when every workgroup streams at once (kLoadedGBs over the
// workgroups that fit, per member): measured alone, a lone workgroup streams
// faster than it can when all of them do.  Then, starting from teams of one,
// the instance whose iteration takes longest gets twice the team while that
// lowers the estimated makespan: the larger of the slowest instance's
// iteration time and the total workgroup time over the workgroups that fit.
constexpr int kProbeIters = 24;
constexpr double kLoadedGBs = 5500.0;   // the batch loops' aggregate rate with every CU busy

struct TuneKey {
  std::string arch;
  int f32, hkind, cls;
  bool operator==(const TuneKey& o) const {
    return arch == o.arch && f32 == o.f32 && hkind == o.hkind && cls == o.cls;
  }
};

static int tune_class(const BInst& I) {
  const double bytes = inst_work(I);
  return std::max(0, (int)std::floor(std::log2(std::max(bytes, 1.0))));
}

// Times one instance alone with one team of g workgroups; us per PCG iteration.
static qp_status probe_team(qp_batch b, int id, int g, const BOpts& bo, double* us) {
  std::vector<int32_t> blob;
  for (int r = 0; r < g; ++r) blob.push_back(0);               // team_of
  const int64_t o_first = (int64_t)blob.size(); blob.push_back(0);
  const int64_t o_size = (int64_t)blob.size(); blob.push_back(g);
  const int64_t o_queue = (int64_t)blob.size(); blob.push_back(0);
  const int64_t o_qstart = (int64_t)blob.size(); blob.push_back(0);
  const int64_t o_qcount = (int64_t)blob.size(); blob.push_back(1);
  const int64_t o_qnext = (int64_t)blob.size(); blob.push_back(0);
  const int64_t o_qorder = (int64_t)blob.size(); blob.push_back(id);
  const int64_t o_abort = (int64_t)blob.size(); blob.push_back(0);
  if ((int64_t)blob.size() > b->plan_cap) {
    if (b->d_plan) (void)hipFree(b->d_plan);
    b->d_plan = nullptr;
    b->plan_cap = 0;
    BCHK(hipMalloc((void**)&b->d_plan, sizeof(int32_t) * blob.size()));
    b->plan_cap = (int64_t)blob.size();
  }
  if (b->sync_cap < 1) {
    BCHK(hipMalloc((void**)&b->d_sync, sizeof(TeamSync)));
    b->sync_cap = 1;
  }
  BCHK(hipMemcpyAsync(b->d_plan, blob.data(), sizeof(int32_t) * blob.size(), hipMemcpyHostToDevice, b->st));
  BCHK(hipMemsetAsync(b->d_sync, 0, sizeof(TeamSync), b->st));
  int32_t* P = b->d_plan;
  TeamPlan plan{};
  plan.team_of = P; plan.first = P + o_first; plan.size = P + o_size; plan.queue = P + o_queue;
  plan.qstart = P + o_qstart; plan.qcount = P + o_qcount; plan.qnext = P + o_qnext;
  plan.qorder = P + o_qorder; plan.sync = b->d_sync; plan.abort = P + o_abort;
  plan.spin_max = team_spin_limit();
  plan.nqueue = 1;
  qp_status ps = ensure_part(b, g);
  if (ps != QP_OK) return ps;
  plan.part = b->d_part;
  plan.ld = b->part_ld;
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  BCHK(hipEventRecord(e0, b->st));
  auto go = [&](auto* tag) -> hipError_t {
    using T = std::remove_pointer_t<decltype(tag)>;
    BArgs<T> a{b->d_inst, b->d_order, b->count, b->d_next, b->d_vec, b->d_out, bo, plan};
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch_ipm<T>), dim3(g), dim3(kBB),
                                      args, 0, b->st);
  };
  BCHK(b->f32 ? go((float*)nullptr) : go((double*)nullptr));
  BCHK(hipEventRecord(e1, b->st));
  BResult r{};
  BCHK(hipMemcpyAsync(&r, b->d_out + id, sizeof(BResult), hipMemcpyDeviceToHost, b->st));
  BCHK(hipStreamSynchronize(b->st));
  float ms = 0.f;
  BCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1e3 * ms / std::max<int64_t>(1, r.total_cg);
  return QP_OK;
}

qp_status qp_batch_autotune(qp_batch b, const char* table_path, int32_t max_team, int32_t* team_out,
                            int32_t* probes_out) {
  if (!b) return QP_ERR_ARG;
  int cap = 0;
  qp_status cs = coresident(b, &cap);
  if (cs != QP_OK) return cs;
  int gmax = max_team > 0 ? std::min(max_team, kTeamMax) : kTeamMax;
  gmax = std::min(gmax, cap);
  int dev = 0;
  hipDeviceProp_t prop;
  BCHK(hipGetDevice(&dev));
  BCHK(hipGetDeviceProperties(&prop, dev));
  std::string arch = prop.gcnArchName;
  for (char& ch : arch) if (ch == ' ') ch = '_';
  // the table: key -> (team size -> us per PCG iteration)
  std::vector<std::pair<TuneKey, std::vector<std::pair<int, double>>>> table;
  auto find = [&](const TuneKey& k) -> std::vector<std::pair<int, double>>* {
    for (auto& e : table) if (e.first == k) return &e.second;
    return nullptr;
  };
  if (table_path) {
    if (FILE* f = std::fopen(table_path, "r")) {
      char a[256];
      int f32, hk, cl, g;
      double us;
      while (std::fscanf(f, "%255s %d %d %d %d %lf", a, &f32, &hk, &cl, &g, &us) == 6) {
        TuneKey k{a, f32, hk, cl};
        auto* v = find(k);
        if (!v) { table.push_back({k, {}}); v = &table.back().second; }
        v->push_back({g, us});
      }
      std::fclose(f);
    }
  }
  BOpts bo{};
  bo.gamma = 0.99; bo.mu0 = 1.0; bo.mu_tol = 1e-6; bo.mu_div = 10.0; bo.max_iter = 1;
  bo.cg_tol = 1e-300; bo.cg_maxit = kProbeIters;
  // representative (largest) instance per class
  std::vector<int> cls(b->count);
  std::vector<std::pair<TuneKey, int>> reps;
  for (int i = 0; i < b->count; ++i) {
    cls[i] = tune_class(b->inst[i]);
    TuneKey k{arch, b->f32 ? 1 : 0, b->inst[i].hkind, cls[i]};
    bool seen = false;
    for (auto& r : reps)
      if (r.first == k) {
        seen = true;
        if (inst_work(b->inst[i]) > inst_work(b->inst[r.second])) r.second = i;
      }
    if (!seen) reps.push_back({k, i});
  }
  int probes = 0;
  std::vector<std::pair<TuneKey, std::pair<int, double>>> fresh;
  for (auto& r : reps) {
    auto* v = find(r.first);
    if (!v) { table.push_back({r.first, {}}); v = &table.back().second; }
    for (int g = 1; g <= gmax; g *= 2) {
      bool have = false;
      for (auto& m : *v) have = have || m.first == g;
      if (have) continue;
      double us = 0.0;
      cs = probe_team(b, r.second, g, bo, &us);
      if (cs != QP_OK) return cs;
      ++probes;
      v->push_back({g, us});
      fresh.push_back({r.first, {g, us}});
    }
  }
  if (table_path && !fresh.empty()) {
    if (FILE* f = std::fopen(table_path, "a")) {
      for (auto& e : fresh)
        std::fprintf(f, "%s %d %d %d %d %.6g\n", e.first.arch.c_str(), e.first.f32, e.first.hkind,
                     e.first.cls, e.second.first, e.second.second);
      std::fclose(f);
    }
  }
  // greedy doubling against the estimated makespan
  auto t_of = [&](int i, int g) -> double {
    TuneKey k{arch, b->f32 ? 1 : 0, b->inst[i].hkind, cls[i]};
    const auto* v = find(k);
    // scale the class's time by this instance's share of its representative's work
    int rep = i;
    for (auto& r : reps) if (r.first == k) rep = r.second;
    const double scale = inst_work(b->inst[i]) / std::max(inst_work(b->inst[rep]), 1e-300);
    const double bytes = inst_work(b->inst[i]) * (b->f32 ? 4.0 : 8.0);
    const double loaded_us = bytes / (g * kLoadedGBs / cap * 1e3);
    for (auto& m : *v) if (m.first == g) return std::max(m.second * scale, loaded_us);
    return INFINITY;
  };
  std::vector<int32_t> team(b->count, 1);
  auto makespan = [&]() {
    double slow = 0.0, total = 0.0;
    for (int i = 0; i < b->count; ++i) {
      const double t = t_of(i, team[i]);
      slow = std::max(slow, t);
      total += t * team[i];
    }
    return std::max(slow, total / cap);
  };
  double cur = makespan();
  for (;;) {
    int worst = -1;
    double tw = -1.0;
    for (int i = 0; i < b->count; ++i) {
      const double t = t_of(i, team[i]);
      if (t > tw) { tw = t; worst = i; }
    }
    if (worst < 0 || team[worst] * 2 > gmax) break;
    team[worst] *= 2;
    const double next = makespan();
    if (!(next < cur)) { team[worst] /= 2; break; }
    cur = next;
  }
  b->team = team;
  b->t_est.assign(b->count, 0.0);
  for (int i = 0; i < b->count; ++i) b->t_est[i] = t_of(i, team[i]);
  if (team_out) std::copy(team.begin(), team.end(), team_out);
  if (probes_out) *probes_out = probes;
  return QP_OK;
}

qp_status qp_batch_set_teams(qp_batch b, const int32_t* team_size) {
  if (!b) return QP_ERR_ARG;
  std::vector<int32_t> t(b->count, 1);
  if (team_size) {
    for (int i = 0; i < b->count; ++i) {
      const int g = team_size[i];
      if (g < 1 || g > kTeamMax || (g & (g - 1))) {
        b->err = "team sizes are powers of two from 1 to " + std::to_string(kTeamMax);
        return QP_ERR_ARG;
      }
      t[i] = g;
    }
  }
  b->team = t;
  b->t_est.clear();
  return QP_OK;
}

qp_status qp_batch_launch_shape(qp_batch b, int32_t* workgroups, int32_t* teams) {
  if (!b) return QP_ERR_ARG;
  if (workgroups) *workgroups = b->last_grid;
  if (teams) *teams = b->last_teams;
  return QP_OK;
}

qp_status qp_batch_instance_times(qp_batch b, double* start_ms, double* end_ms, int32_t* team) {
  if (!b) return QP_ERR_ARG;
  if (!b->have_out) {
    b->err = "no completed ipm_solve_batch on this batch yet";
    return QP_ERR_ARG;
  }
  int dev = 0, khz = 0;
  BCHK(hipGetDevice(&dev));
  BCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) {
    b->err = "the device reports no wall clock rate";
    return QP_ERR_HIP;
  }
  int64_t t0 = INT64_MAX;
  for (const BResult& r : b->out) t0 = std::min(t0, r.t_start);
  for (int i = 0; i < b->count; ++i) {
    const BResult& r = b->out[i];
    if (start_ms) start_ms[i] = static_cast<double>(r.t_start - t0) / khz;
    if (end_ms) end_ms[i] = static_cast<double>(r.t_end - t0) / khz;
    if (team) team[i] = r.team;
  }
  return QP_OK;
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
