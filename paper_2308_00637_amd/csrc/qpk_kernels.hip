// Device kernels of libqpk for gfx950 (CDNA4, wave64).
//
// The doubly augmented matrix of eq. (9) (Section 3.1),
//     K = [[Q + 2 B^T D^-1 B, B^T], [B, D]],  B = [C; A_L; -A_U],
// is applied matrix-free (Section 3.2).  For a K-vector v = (v_x, v_e, v_l, v_u):
//     t = B v_x,  y_lam = t + D v_lam,  w = 2 D^-1 t + v_lam,
//     y_x = H v_x + q_b * v_x + B^T w.
// Row i of A contributes t_i = A_i . v_x and then A_i^T (w_l,i - w_u,i) to y_x,
// so the work splits into a row-side pass (one segmented dot per row of A, and
// per row of P when H = P^T W P) and a column-side pass over the transposed
// operators (one segmented dot per variable).  Every reduction below has a
// fixed order (lane tree, then block tree, then blocks in index order), so a
// run is bitwise reproducible.
#include "qpk_internal.h"

#include <math.h>

namespace qpk {

// ------------------------------------------------------------------ basics
template <int VK> struct VT;
template <> struct VT<VK_F64> { using T = double;   using Acc = double; };
template <> struct VT<VK_F32> { using T = float;    using Acc = float; };
template <> struct VT<VK_BF16> { using T = uint16_t; using Acc = float; };
template <> struct VT<VK_F32X> { using T = float;    using Acc = double; };
template <> struct VT<VK_BF16X> { using T = uint16_t; using Acc = double; };

__device__ __forceinline__ double ldv(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const uint16_t* p, int64_t i) {
  return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}

typedef __attribute__((address_space(1))) void gvoid;   // global memory
typedef __attribute__((address_space(3))) void lvoid;   // LDS

// Two consecutive stored values from an even (pair-aligned) index: one 16-,
// 8- or 4-byte load.
__device__ __forceinline__ void ldv2(const double* p, int64_t i, double& x, double& y) {
  const double2 v = *reinterpret_cast<const double2*>(p + i);
  x = v.x;
  y = v.y;
}
__device__ __forceinline__ void ldv2(const float* p, int64_t i, float& x, float& y) {
  const float2 v = *reinterpret_cast<const float2*>(p + i);
  x = v.x;
  y = v.y;
}
__device__ __forceinline__ void ldv2(const uint16_t* p, int64_t i, float& x, float& y) {
  const uint32_t u = *reinterpret_cast<const uint32_t*>(p + i);
  x = __uint_as_float(u << 16);
  y = __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ bool has_lo(double l) { return l > -INFINITY; }
__device__ __forceinline__ bool has_hi(double u) { return u < INFINITY; }

template <int W, typename A>
__device__ __forceinline__ A group_sum(A v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// Sum over the block; the result is valid on thread 0.
__device__ double block_sum(double v) {
  __shared__ double sh[kBlock / 64];
  v = group_sum<64>(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

__device__ double block_min(double v) {
  __shared__ double sh[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = INFINITY;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) r = fmin(r, sh[i]);
  }
  __syncthreads();
  return r;
}

// Sum of cnt partials, identical on every thread of the block.
__device__ double sum_bcast(const double* p, int cnt) {
  __shared__ double shb;
  double v = 0.0;
  for (int i = threadIdx.x; i < cnt; i += kBlock) v += p[i];
  v = block_sum(v);
  if (threadIdx.x == 0) shb = v;
  __syncthreads();
  v = shb;
  __syncthreads();
  return v;
}

// Three block-wide sums of per-block partials, broadcast to every thread.
// Each sum runs in the same order as sum_bcast (thread-strided, then the block
// tree), so the results are bitwise those of three sum_bcast calls; the three
// partial arrays are read together, so the block waits for one latency.
__device__ void sum3_bcast(const double* p0, int c0, const double* p1, int c1, const double* p2,
                           int c2, double& s0, double& s1, double& s2) {
  __shared__ double sh[3][kBlock / 64];
  __shared__ double out[3];
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int i = threadIdx.x; i < c0; i += kBlock) v0 += p0[i];
  for (int i = threadIdx.x; i < c1; i += kBlock) v1 += p1[i];
  for (int i = threadIdx.x; i < c2; i += kBlock) v2 += p2[i];
  v0 = group_sum<64>(v0);
  v1 = group_sum<64>(v1);
  v2 = group_sum<64>(v2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = v0;
    sh[1][w] = v1;
    sh[2][w] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) r += sh[threadIdx.x][i];
    out[threadIdx.x] = r;
  }
  __syncthreads();
  s0 = out[0];
  s1 = out[1];
  s2 = out[2];
}

__device__ double min_bcast(const double* p, int cnt) {
  __shared__ double shb;
  double v = INFINITY;
  for (int i = threadIdx.x; i < cnt; i += kBlock) v = fmin(v, p[i]);
  v = block_min(v);
  if (threadIdx.x == 0) shb = v;
  __syncthreads();
  v = shb;
  __syncthreads();
  return v;
}

// Offsets into the residual stack.
struct ResOff {
  int64_t rH, re, rlA, ruA, rlx, rux, rc1, rc2, rc3, rc4;
  __device__ ResOff(int n, int m, int me) {
    rH = 0; re = n; rlA = re + me; ruA = rlA + m; rlx = ruA + m; rux = rlx + n;
    rc1 = rux + n; rc2 = rc1 + m; rc3 = rc2 + m; rc4 = rc3 + n;
  }
};

// ------------------------------------------------------- row-side pass
// One group of LPR lanes per row of RP (rows of P, then rows of A).
template <int MODE, int VK, int LPR>
__global__ __launch_bounds__(kBlock) void k_rowpass(RowArgs a) {
  using T = typename VT<VK>::T;
  using Acc = typename VT<VK>::Acc;
  if (a.done && *a.done) return;
  const T* __restrict__ val = static_cast<const T*>(a.val);
  const int lane = threadIdx.x & (LPR - 1);
  const int gid = (blockIdx.x * kBlock + threadIdx.x) / LPR;
  const int ng = gridDim.x * (kBlock / LPR);
  const int n = a.n, m = a.m, me = a.me;
  double acc0 = 0.0, acc1 = 0.0;
  double mn0 = INFINITY, mn1 = INFINITY;
  for (int row = a.r0 + gid; row < a.r1; row += ng) {
    const int beg = a.rowptr[row], end = a.rowptr[row + 1];
    Acc t = 0, t2 = 0;
    for (int q = beg + lane; q < end; q += LPR) {
      const int c = a.col[q];
      const Acc vv = ldv(val, q);
      t += vv * static_cast<Acc>(a.v[c]);
      if constexpr (MODE == R_GRADW) t2 += vv * static_cast<Acc>(a.v2[c]);
    }
    t = group_sum<LPR>(t);
    if constexpr (MODE == R_GRADW) t2 = group_sum<LPR>(t2);
    if (lane != 0) continue;
    const double td = static_cast<double>(t);
    if (row < a.p_rows) {
      if constexpr (MODE == R_MATVEC || MODE == R_RESID || MODE == R_PU) {
        a.u[row] = a.w[row] * td;
      } else if constexpr (MODE == R_GRADW) {
        const double dv = a.d ? a.d[row] : 0.0;
        a.gw[row] = -td * (static_cast<double>(t2) - dv);
      }
      continue;
    }
    const int i = row - a.p_rows;
    const bool hl = has_lo(a.lA[i]), hu = has_hi(a.uA[i]);
    if constexpr (MODE == R_MATVEC) {
      const double vlo = a.vl[me + i], vup = a.vl[me + m + i];
      const double dlo = a.dl[me + i], dup = a.dl[me + m + i];
      const double ylo = (hl ? td : 0.0) + dlo * vlo;
      const double yup = (hu ? -td : 0.0) + dup * vup;
      a.yl[me + i] = ylo;
      a.yl[me + m + i] = yup;
      a.wA[i] = (hl ? 2.0 * td / dlo + vlo : 0.0) - (hu ? -2.0 * td / dup + vup : 0.0);
      acc0 += vlo * ylo + vup * yup;
    } else if constexpr (MODE == R_RESID) {
      const ResOff o(n, m, me);
      const double ll = a.lam[me + i], lu = a.lam[me + m + i];
      const double sl = a.s[i], su = a.s[m + i];
      const double rl = hl ? td - sl - a.lA[i] : 0.0;
      const double ru = hu ? -td - su + a.uA[i] : 0.0;
      const double c1 = hl ? ll * sl - a.tau : 0.0;
      const double c2 = hu ? lu * su - a.tau : 0.0;
      a.resw[o.rlA + i] = rl;
      a.resw[o.ruA + i] = ru;
      a.resw[o.rc1 + i] = c1;
      a.resw[o.rc2 + i] = c2;
      a.wA[i] = (hu ? lu : 0.0) - (hl ? ll : 0.0);
      acc0 += rl * rl + ru * ru;
      acc1 += c1 * c1 + c2 * c2;
    } else if constexpr (MODE == R_RECOVER) {
      const ResOff o(n, m, me);
      const double dsl = hl ? td + a.res[o.rlA + i] : 0.0;
      const double dsu = hu ? -td + a.res[o.ruA + i] : 0.0;
      a.ds[i] = dsl;
      a.ds[m + i] = dsu;
      const double dll = a.dlam[me + i], dlu = a.dlam[me + m + i];
      if (hl && dsl < 0.0) mn0 = fmin(mn0, -a.s[i] / dsl);
      if (hu && dsu < 0.0) mn0 = fmin(mn0, -a.s[m + i] / dsu);
      if (hl && dll < 0.0) mn1 = fmin(mn1, -a.lam[me + i] / dll);
      if (hu && dlu < 0.0) mn1 = fmin(mn1, -a.lam[me + m + i] / dlu);
    } else if constexpr (MODE == R_INIT) {
      a.ds[i] = hl ? fmax(td - a.lA[i], 1.0) : 0.0;          // ds aliases s here
      a.ds[m + i] = hu ? fmax(a.uA[i] - td, 1.0) : 0.0;
      a.yl[me + i] = hl ? 1.0 : 0.0;                          // yl aliases lam here
      a.yl[me + m + i] = hu ? 1.0 : 0.0;
    }
  }
  if constexpr (MODE == R_MATVEC || MODE == R_RESID) {
    const double s0 = block_sum(acc0);
    const double s1 = block_sum(acc1);
    if (threadIdx.x == 0) {
      a.part0[blockIdx.x] = s0;
      if (a.part1) a.part1[blockIdx.x] = s1;
    }
  } else if constexpr (MODE == R_RECOVER) {
    const double s0 = block_min(mn0);
    const double s1 = block_min(mn1);
    if (threadIdx.x == 0) {
      a.part0[blockIdx.x] = s0;
      a.part1[blockIdx.x] = s1;
    }
  }
}

// ---------------------------------------------------- column-side pass
// One group of LPR lanes per variable j: segments of XS row j, the low-rank
// row U_j, the equality columns C_:j, then a per-mode epilogue.
template <int MODE, int VK, int LPR>
__global__ __launch_bounds__(kBlock) void k_colpass(ColArgs a) {
  using T = typename VT<VK>::T;
  using Acc = typename VT<VK>::Acc;
  if (a.done && *a.done) return;
  if (a.bump && blockIdx.x == 0 && threadIdx.x == 0) *a.bump += 1;
  const T* __restrict__ val = static_cast<const T*>(a.val);
  const T* __restrict__ U = static_cast<const T*>(a.U);
  const int lane = threadIdx.x & (LPR - 1);
  const int gid = (blockIdx.x * kBlock + threadIdx.x) / LPR;
  const int ng = gridDim.x * (kBlock / LPR);
  const int n = a.n, m = a.m, me = a.me, k = a.k;
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  // X_MATVEC: lane s of a group keeps the dot of the group's s-th row; every
  // LPR rows, and after the last, each lane runs the epilogue of the row it
  // holds, so the stores leave in bursts instead of one per row between the
  // loads (21% off U(w g) on a 500k x 128 factor).
  int held_n = 0, held_j = 0;
  double held = 0.0;
  auto flush = [&]() {
    if (lane < held_n) {
      double y = held;
      for (int e = 0; e < me; ++e) y += a.Cm[static_cast<int64_t>(e) * n + held_j] * a.we[e];
      const double vj = a.v[held_j];
      y += a.qdiag[held_j] * vj;
      a.y[held_j] = y;
      p0 += vj * y;
    }
    held_n = 0;
  };
  // Products with a low-rank H and no stored segments (the SVM form): four
  // rows per group in flight.
  bool rows_done = false;
  if constexpr (MODE == X_MATVEC) {
    if (!val && k > 0) {
      rows_done = true;
      constexpr int R = 4;
      using LT = decltype(ldv(U, 0));
      for (int j0 = gid; j0 < n; j0 += R * ng) {
        Acc acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int j = j0 + r * ng;
          acc[r] = 0;
          if (j < n) {
            const int64_t base = static_cast<int64_t>(j) * k;
            if ((k & 1) == 0) {
              // even k: rows start pair-aligned, one 16-byte (float64) load per pair
#pragma unroll 2
              for (int l = 2 * lane; l < k; l += 2 * LPR) {
                LT ux, uy;
                ldv2(U, base + l, ux, uy);
                acc[r] += static_cast<Acc>(ux) * static_cast<Acc>(a.g[l]);
                acc[r] += static_cast<Acc>(uy) * static_cast<Acc>(a.g[l + 1]);
              }
            } else {
#pragma unroll 4
              for (int l = lane; l < k; l += LPR) acc[r] += ldv(U, base + l) * static_cast<Acc>(a.g[l]);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = group_sum<LPR>(acc[r]);   // butterfly: on every lane
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int j = j0 + r * ng;
          if (j < n) {
            if (lane == held_n) {
              held = static_cast<double>(acc[r]);
              held_j = j;
            }
            if (++held_n == LPR) flush();
          }
        }
      }
    }
  }
  if (!rows_done)
  for (int j = gid; j < n; j += ng) {
    Acc acc = 0, acc2 = 0;
    if (val) {
      const int b0 = a.rowptr[j], b1 = a.seg1[j], b2 = a.seg2[j], b3 = a.rowptr[j + 1];
      // unrolled so that each lane has several entries' loads in flight
      // (same summation order)
      if (MODE != X_RHS && MODE != X_DIAGH && MODE != X_CEFF && a.use_hx) {
#pragma unroll 8
        for (int q = b0 + lane; q < b1; q += LPR)
          acc += ldv(val, q) * static_cast<Acc>(a.src_hx[a.col[q]]);
      }
      if (a.use_pt) {
#pragma unroll 4
        for (int q = b1 + lane; q < b2; q += LPR) {
          const int c = a.col[q];
          const Acc vv = ldv(val, q);
          if constexpr (MODE == X_DIAGH) acc += vv * vv * static_cast<Acc>(a.w[c]);
          else if constexpr (MODE == X_CEFF) acc += vv * static_cast<Acc>(a.w[c] * a.src_pt[c]);
          else acc += vv * static_cast<Acc>(a.src_pt[c]);
        }
      }
      if (a.use_at) {
#pragma unroll 4
        for (int q = b2 + lane; q < b3; q += LPR) {
          const int c = a.col[q];
          const Acc vv = ldv(val, q);
          acc += vv * static_cast<Acc>(a.src_at[c]);
          if constexpr (MODE == X_RHS) acc2 += vv * vv * static_cast<Acc>(a.src_at2[c]);
        }
      }
    }
    if constexpr (MODE == X_MATVEC || MODE == X_RESID || MODE == X_OBJ || MODE == X_DIAGH) {
      if (k > 0) {
        const int64_t base = static_cast<int64_t>(j) * k;
        for (int l = lane; l < k; l += LPR) {
          const Acc uv = ldv(U, base + l);
          if constexpr (MODE == X_DIAGH) acc += uv * uv * static_cast<Acc>(a.wd[l]);
          else acc += uv * static_cast<Acc>(a.g[l]);
        }
      }
    }
    acc = group_sum<LPR>(acc);   // butterfly: on every lane
    if constexpr (MODE == X_RHS) acc2 = group_sum<LPR>(acc2);
    if constexpr (MODE == X_MATVEC) {
      if (lane == held_n) {
        held = static_cast<double>(acc);
        held_j = j;
      }
      if (++held_n == LPR) flush();
      continue;
    }
    if (lane != 0) continue;
    double y = static_cast<double>(acc);
    if constexpr (MODE == X_RESID) {
      const ResOff o(n, m, me);
      const double xj = a.v[j];
      for (int e = 0; e < me; ++e) y += a.Cm[static_cast<int64_t>(e) * n + j] * a.we[e];
      if (a.h0) y += a.h0[j] * xj;
      y += a.c[j];
      const bool hl = has_lo(a.lx[j]), hu = has_hi(a.ux[j]);
      const double llx = hl ? a.lam[me + 2 * m + j] : 0.0;
      const double lux = hu ? a.lam[me + 2 * m + n + j] : 0.0;
      const double slx = a.s[2 * m + j], sux = a.s[2 * m + n + j];
      y += -llx + lux;
      const double rlx = hl ? xj - slx - a.lx[j] : 0.0;
      const double rux = hu ? -xj - sux + a.ux[j] : 0.0;
      const double c3 = hl ? llx * slx - a.tau : 0.0;
      const double c4 = hu ? lux * sux - a.tau : 0.0;
      a.res[o.rH + j] = y;
      a.res[o.rlx + j] = rlx;
      a.res[o.rux + j] = rux;
      a.res[o.rc3 + j] = c3;
      a.res[o.rc4 + j] = c4;
      p0 += y * y;
      p1 += rlx * rlx + rux * rux;
      p2 += c3 * c3 + c4 * c4;
    } else if constexpr (MODE == X_RHS) {
      const ResOff o(n, m, me);
      const bool hl = has_lo(a.lx[j]), hu = has_hi(a.ux[j]);
      const double llx = hl ? a.lam[me + 2 * m + j] : 0.0;
      const double lux = hu ? a.lam[me + 2 * m + n + j] : 0.0;
      const double slx = hl ? a.s[2 * m + j] : 1.0, sux = hu ? a.s[2 * m + n + j] : 1.0;
      const double rH = a.res_in[o.rH + j];
      const double rlx = a.res_in[o.rlx + j], rux = a.res_in[o.rux + j];
      const double c3 = a.res_in[o.rc3 + j], c4 = a.res_in[o.rc4 + j];
      const double qb = (hl ? llx / slx : 0.0) + (hu ? lux / sux : 0.0);
      double r1 = -rH;
      if (hl) r1 += -c3 / slx - llx / slx * rlx;
      if (hu) r1 += c4 / sux + lux / sux * rux;
      double top = r1 + y;
      double jd = a.diagH[j] + qb + static_cast<double>(acc2);
      for (int e = 0; e < me; ++e) {
        const double cej = a.Cm[static_cast<int64_t>(e) * n + j];
        top += cej * a.we[e];
        jd += 2.0 * cej * cej / a.mu;
      }
      a.rhs[j] = top;
      a.jdiag[j] = jd;
      a.qdiag_out[j] = (a.h0 ? a.h0[j] : 0.0) + qb;
    } else if constexpr (MODE == X_DIAGH) {
      a.y[j] = a.v[j] + y;
    } else if constexpr (MODE == X_CEFF) {
      a.y[j] = a.c[j] - y;
    } else if constexpr (MODE == X_OBJ) {
      const double xj = a.v[j];
      if (a.h0) y += a.h0[j] * xj;
      p0 += xj * (0.5 * y + a.c[j]);
    }
  }
  if constexpr (MODE == X_MATVEC) flush();
  if constexpr (MODE == X_MATVEC || MODE == X_RESID || MODE == X_OBJ) {
    const double s0 = block_sum(p0);
    double s1 = 0.0, s2 = 0.0;
    if constexpr (MODE == X_RESID) {
      s1 = block_sum(p1);
      s2 = block_sum(p2);
    }
    if (threadIdx.x == 0) {
      a.part0[blockIdx.x] = s0;
      if constexpr (MODE == X_RESID) {
        a.part1[blockIdx.x] = s1;
        a.part2[blockIdx.x] = s2;
      }
    }
  }
}

// ------------------------------------------------ matvec epilogues
// Matvec epilogues shared by the PCG passes.
// Epilogue of A row i with dot td: its y_lam entries and wA_i (also returned
// in wa); returns its term of v_lam . (K v)_lam, plus with a.xdot t_i wA_i.
__device__ __forceinline__ double a_row_epilogue(const RowArgs& a, int i, double td, double& wa) {
  const int me = a.me, m = a.m;
  const bool hl = has_lo(a.lA[i]), hu = has_hi(a.uA[i]);
  const double vlo = a.vl[me + i], vup = a.vl[me + m + i];
  const double dlo = a.dl[me + i], dup = a.dl[me + m + i];
  const double ylo = (hl ? td : 0.0) + dlo * vlo;
  const double yup = (hu ? -td : 0.0) + dup * vup;
  a.yl[me + i] = ylo;
  a.yl[me + m + i] = yup;
  wa = (hl ? 2.0 * td / dlo + vlo : 0.0) - (hu ? -2.0 * td / dup + vup : 0.0);
  a.wA[i] = wa;
  return vlo * ylo + vup * yup + (a.xdot ? td * wa : 0.0);
}

// Row epilogue of the PCG matvec (R_MATVEC): P rows give u = w t; A rows give
// the lam-part of K v and wA = w_l - w_u.  Returns this row's term of
// v_lam . (K v)_lam, plus with a.xdot its term of v_x . (K v)_x:
// v_x . P^T u = sum_v t_v u_v and v_x . A^T wA = sum_i t_i wA_i.
// With a.twin, a P row that an A row repeats also runs that A row's epilogue
// on its own dot, and stores u + wA: the column pass, which then holds P^T
// alone, multiplies by it (P^T u + A^T wA = P^T (u + S wA), S the twin map).
__device__ __forceinline__ double row_matvec_epilogue(const RowArgs& a, int row, double td) {
  if (row < a.p_rows) {
    const double uv = a.w[row] * td;
    double dot = a.xdot ? td * uv : 0.0;
    double ut = uv;
    if (a.twin) {
      const int i = a.twin[row];
      if (i >= 0) {
        double wa;
        dot += a_row_epilogue(a, i, td, wa);
        ut += wa;
      }
    }
    a.u[row] = ut;
    return dot;
  }
  double wa;
  return a_row_epilogue(a, row - a.p_rows, td, wa);
}

// Column epilogue of the PCG matvec (X_MATVEC); returns v_j y_j.
__device__ __forceinline__ double col_matvec_epilogue(const ColArgs& a, int j, double y) {
  for (int e = 0; e < a.me; ++e) y += a.Cm[static_cast<int64_t>(e) * a.n + j] * a.we[e];
  const double vj = a.v[j];
  y += a.qdiag[j] * vj;
  a.y[j] = y;
  return vj * y;
}

// ------------------------------------------- LDS-staged blocked passes
template <int NT>
__device__ double block_sum_nt(double v) {
  __shared__ double sh[NT / 64];
  v = group_sum<64>(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// Bijection of [0, g): the blocks i with i mod 8 == x map to the x-th
// contiguous run of items.
__device__ __forceinline__ int xcd_item(int i, int g) {
  const int x = i & 7, slot = i >> 3, q = g >> 3, r = g & 7;
  return x * q + min(x, r) + slot;
}

// Raw buffer resources: a load whose byte offset is at or past num_records
// returns zero without touching memory, so loads past a segment's end need no
// branch.  kOob is such an offset for every array here (all are < 2 GiB).
constexpr uint32_t kOob = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;   // 32-bit data format, no swizzle
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), kRsrcWord3);
}
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef int i2v __attribute__((ext_vector_type(2)));

// A value pair at byte offset o (zero when o is out of range).
__device__ __forceinline__ void ldv2b(const double*, __amdgpu_buffer_rsrc_t r, uint32_t o, double& x,
                                      double& y) {
  const d2v v = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0));
  x = v.x;
  y = v.y;
}
__device__ __forceinline__ void ldv2b(const float*, __amdgpu_buffer_rsrc_t r, uint32_t o, float& x,
                                      float& y) {
  const f2v v = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
  x = v.x;
  y = v.y;
}
__device__ __forceinline__ void ldv2b(const uint16_t*, __amdgpu_buffer_rsrc_t r, uint32_t o, float& x,
                                      float& y) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0);
  x = __uint_as_float(u << 16);
  y = __uint_as_float(u & 0xffff0000u);
}

// This thread's lane in its wave, recomputed where it is called: the rare
// rows longer than one batch take their lane offsets from it, so the column
// pass (held to 64 VGPRs) need not keep them live across the row loop, which
// had cost three spilled registers per thread.
__device__ __forceinline__ int lane_of_wave() {
  int r;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(r));
  return r;
}

// Kernel variants: KV 0 stages the chunk through registers (16-byte loads,
// all issued at once), KV 1 with direct global-to-LDS loads (no registers
// held, so a half-LDS chunk pass fits 64 VGPRs and two blocks share a CU).
//
// Every (chunk, row) segment starts at an even entry and has even length
// (zero-padded), so a lane loads its entries in pairs: one 16-byte value load
// (float64) and one 4-byte load of two uint16 column offsets per pair.  A
// group of LPR lanes reduces one row; lane l takes pairs l, l + LPR, ...
template <int EPI, int VK, int LPR, int KV>
__device__ __forceinline__ void chunked_body(const ChunkArgs& b, const RowArgs& ra, const ColArgs& ca) {
  using T = typename VT<VK>::T;
  using Acc = typename VT<VK>::Acc;
  constexpr bool DMA = KV == 1;
  if ((ra.done && *ra.done) || (ca.done && *ca.done)) return;
  if constexpr (EPI != CE_ROW) {
    if (ca.bump && blockIdx.x == 0 && threadIdx.x == 0) *ca.bump += 1;
  }
  extern __shared__ __align__(16) double lds[];
  // Work items are stored chunk by chunk.  Blocks go to the 8 XCDs round
  // robin (block i on XCD i mod 8), so block i takes item xcd_item(i): the
  // blocks of one XCD take a contiguous run of items, i.e. a few chunks, whose
  // gathered vector its own L2 then fetches once.
  const int wi = b.xcd_map ? xcd_item(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
  const int c = b.work[3 * wi], r0 = b.work[3 * wi + 1], r1 = b.work[3 * wi + 2];
  const int32_t* rp = b.rowptr + static_cast<int64_t>(c) * (b.nrows + 1);
  const T* val = static_cast<const T*>(b.val);
  const __amdgpu_buffer_rsrc_t rrp = rsrc(rp, 4u * static_cast<uint32_t>(b.nrows + 1));
  const __amdgpu_buffer_rsrc_t rcol = rsrc(b.col, 2u * static_cast<uint32_t>(b.nstored));
  const __amdgpu_buffer_rsrc_t rval = rsrc(val, static_cast<uint32_t>(sizeof(T)) * b.nstored);
  const int lane = threadIdx.x & (LPR - 1);
  const int gid = threadIdx.x / LPR;
  constexpr int NG = kChunkBlock / LPR;
  // entry pairs per lane per batch: a pass staged through registers runs one
  // block per CU (a full-LDS chunk), so up to 128 VGPRs, and takes eight at
  // up to 8 lanes per row, twice the entries in flight per wave
  constexpr int PP = (!DMA && LPR <= 8) ? 8 : 4;
  constexpr int SPAN = 2 * LPR * PP;         // entries per group per batch
  using LT = decltype(ldv(val, 0));          // loaded value type

  // the pairs of one batch starting at entry `base` of a segment ending at `end`
  auto load_batch = [&](int base, int end, uint32_t* cc, LT* vx, LT* vy, int ln) {
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      const int q = base + 2 * (ln + k * LPR);
      const bool ok = q < end;
      cc[k] = __builtin_amdgcn_raw_buffer_load_b32(rcol, ok ? 2u * q : kOob, 0, 0);
      ldv2b(val, rval, ok ? static_cast<uint32_t>(sizeof(T)) * q : kOob, vx[k], vy[k]);
    }
  };
  // [rowptr[r], rowptr[r + 1]) for r < r1, else an empty segment
  // This group's rows are r0 + gid + k NG, k = 0 .. nk-1, visited in that order
  // or (b.reverse) mirrored within [r0, r1), last row first.  Alternating the
  // direction between passes starts each pass on the data the previous pass
  // over the same operator touched last, which the memory-side cache still holds.
  const int nk = r1 - r0 > gid ? (r1 - r0 - gid + NG - 1) / NG : 0;
  auto row_of = [&](int k) { return b.reverse ? r1 - 1 - gid - k * NG : r0 + gid + k * NG; };
  auto bounds = [&](int k, int& beg, int& end) {
    const i2v be = __builtin_bit_cast(
        i2v, __builtin_amdgcn_raw_buffer_load_b64(rrp, k < nk ? 4u * row_of(k) : kOob, 0, 0));
    beg = be.x;
    end = be.y;
  };

  const int c0 = c * b.chunk_cols;
  const int cw = min(b.chunk_cols, b.ncols - c0);
  constexpr int SP = DMA ? 1 : (kChunkCols + 2 * kChunkBlock - 1) / (2 * kChunkBlock);
  double2 st[SP];
  if constexpr (DMA) {
    // wave w copies the 1 KB pieces w, w + 16, ... of the chunk, 16 bytes a lane
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int npair = cw >> 1;
    for (int base = wv * 64; base < npair; base += kChunkBlock) {
      if (base + ln < npair)
        __builtin_amdgcn_global_load_lds((gvoid*)(b.src + c0 + 2 * (base + ln)),
                                         (lvoid*)(lds + 2 * base), 16, 0, 0);
    }
  } else {
    // every staging load at once, so the block waits for one memory latency
    const __amdgpu_buffer_rsrc_t rsv = rsrc(b.src + c0, 16u * static_cast<uint32_t>(cw >> 1));
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const uint32_t i2 = threadIdx.x + k * kChunkBlock;
      st[k] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rsv, 16u * i2, 0, 0));
    }
  }
  // Software pipeline over this group's rows r0 + gid, + NG, ...: the row
  // bounds are loaded three rows ahead and the entry batch one row ahead of
  // the row being reduced, so no load waits on another's latency.
  int beg, end, b1, e1, b2, e2;
  bounds(0, beg, end);
  bounds(1, b1, e1);
  bounds(2, b2, e2);
  uint32_t cc[PP], cc1[PP];
  LT vx[PP], vy[PP], vx1[PP], vy1[PP];
  load_batch(beg, end, cc, vx, vy, lane);
  if constexpr (DMA) {
    __builtin_amdgcn_s_waitcnt(0);   // LDS-direct loads are counted as vector loads
  } else {
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int i2 = threadIdx.x + k * kChunkBlock;
      if (2 * i2 + 1 < cw) reinterpret_cast<double2*>(lds)[i2] = st[k];
    }
  }
  if ((cw & 1) && threadIdx.x == 0) lds[cw - 1] = b.src[c0 + cw - 1];
  __syncthreads();

  double acc0 = 0.0;
  double held = 0.0;
  for (int kr = 0; kr < nk; ++kr) {
    int b3, e3;
    bounds(kr + 3, b3, e3);
    load_batch(b1, e1, cc1, vx1, vy1, lane);
    Acc t = 0;
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      t += static_cast<Acc>(vx[k]) * static_cast<Acc>(lds[cc[k] & 0xffffu]);
      t += static_cast<Acc>(vy[k]) * static_cast<Acc>(lds[cc[k] >> 16]);
    }
    for (int base = beg + SPAN; base < end; base += SPAN) {   // rows longer than one batch
      uint32_t c2[PP];
      LT x[PP], y[PP];
      load_batch(base, end, c2, x, y, lane_of_wave() & (LPR - 1));
#pragma unroll
      for (int k = 0; k < PP; ++k) {
        t += static_cast<Acc>(x[k]) * static_cast<Acc>(lds[c2[k] & 0xffffu]);
        t += static_cast<Acc>(y[k]) * static_cast<Acc>(lds[c2[k] >> 16]);
      }
    }
    t = group_sum<LPR>(t);   // butterfly: every lane of the group holds the same sum
    // Lane kr mod LPR keeps this row's dot; every LPR rows, and after the
    // group's last row, each lane runs the epilogue of the row it holds.  A
    // pass with at most LPR rows per group thus issues all of its stores at
    // the end, instead of one small store per row between the loads, which
    // measured ~3 us (6%) faster on a cold-cache 210 MB pass.
    const int slot = kr & (LPR - 1);
    if (lane == slot) held = static_cast<double>(t);
    if (slot == LPR - 1 || kr == nk - 1) {
      const int k = kr - slot + lane;
      if (k <= kr) {
        const int hrow = row_of(k);
        if constexpr (EPI == CE_PARTIAL) {
          b.partial[static_cast<int64_t>(c) * b.nrows + hrow] = held;
        } else if constexpr (EPI == CE_ROW) acc0 += row_matvec_epilogue(ra, hrow, held);
        else acc0 += col_matvec_epilogue(ca, hrow, held);
      }
    }
    beg = b1;
    end = e1;
    b1 = b2;
    e1 = e2;
    b2 = b3;
    e2 = e3;
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      cc[k] = cc1[k];
      vx[k] = vx1[k];
      vy[k] = vy1[k];
    }
  }
  // ra.xdot: the terms of v_x . (K v)_x that are not row terms (equality rows,
  // diagonal), block b taking the b-th slice of x; v_x is the staged chunk
  if (EPI == CE_ROW && ra.xdot) {
    const int j0 = static_cast<int>(static_cast<int64_t>(ra.n) * blockIdx.x / gridDim.x);
    const int j1 = static_cast<int>(static_cast<int64_t>(ra.n) * (blockIdx.x + 1) / gridDim.x);
    for (int j = j0 + threadIdx.x; j < j1; j += kChunkBlock) {
      const double vj = lds[j];
      double e = 0.0;
      for (int i = 0; i < ra.me; ++i) e += ra.Cm[static_cast<int64_t>(i) * ra.n + j] * ra.we[i];
      acc0 += vj * e + ra.qdiag[j] * vj * vj;
    }
  }
  if constexpr (EPI != CE_PARTIAL) {
    acc0 = block_sum_nt<kChunkBlock>(acc0);
    if (threadIdx.x == 0) {
      if constexpr (EPI == CE_ROW) ra.part0[blockIdx.x] = acc0;
      else ca.part0[blockIdx.x] = acc0;
    }
  }
}

// Waves per SIMD the compiler must leave room for: a multi-chunk pass without
// register staging is held to 64 VGPRs so two 1024-thread blocks share a CU.
template <int EPI, int KV>
constexpr int chunked_min_waves() { return (EPI == CE_PARTIAL && KV == 1) ? 8 : 1; }

template <int EPI, int VK, int LPR, int KV>
__global__ __launch_bounds__(kChunkBlock)
__attribute__((amdgpu_waves_per_eu(chunked_min_waves<EPI, KV>())))
void k_chunked(ChunkArgs b, RowArgs ra, ColArgs ca) {
  chunked_body<EPI, VK, LPR, KV>(b, ra, ca);
}

// Sum of the per-chunk partials, then the matvec epilogue.  The chunks are
// cut into four consecutive groups of ceil(nchunk / 4); each group is summed
// in chunk order from 0.0 and the four sums are combined as (g0 + g1) +
// (g2 + g3).  The PCG update sums the x-part of q in exactly this order, one
// group per quarter of a wave, so q is bitwise the same either way.
__device__ __forceinline__ int partial_group(int nchunk) { return (nchunk + 3) >> 2; }

__device__ __forceinline__ double sum_partials(const ChunkArgs& b, int r) {
  const double* p = b.partial + r;
  const int64_t st = b.nrows;
  const int g = partial_group(b.nchunk);
  double y[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int c1 = min(b.nchunk, (s + 1) * g);
    double acc = 0.0;
    int c = s * g;
    for (; c + 8 <= c1; c += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = p[(c + u) * st];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += t[u];
    }
    for (; c < c1; ++c) acc += p[c * st];
    y[s] = acc;
  }
  return (y[0] + y[1]) + (y[2] + y[3]);
}

__global__ __launch_bounds__(kBlock) void k_chunk_epilogue_col(ChunkArgs b, ColArgs a) {
  if (a.done && *a.done) return;
  if (a.bump && blockIdx.x == 0 && threadIdx.x == 0) *a.bump += 1;
  double acc0 = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < b.nrows; j += gridDim.x * kBlock)
    acc0 += col_matvec_epilogue(a, j, sum_partials(b, j));
  acc0 = block_sum(acc0);
  if (threadIdx.x == 0) a.part0[blockIdx.x] = acc0;
}

__global__ __launch_bounds__(kBlock) void k_chunk_epilogue_row(ChunkArgs b, RowArgs a) {
  if (a.done && *a.done) return;
  double acc0 = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < b.nrows; r += gridDim.x * kBlock)
    acc0 += row_matvec_epilogue(a, r, sum_partials(b, r));
  acc0 = block_sum(acc0);
  if (threadIdx.x == 0) a.part0[blockIdx.x] = acc0;
}

// ------------------------------------------ fused single-read PCG product
// For H = P^T W P every row of the row operator (rows of P, then rows of A,
// or P alone with its twin map) contributes RP_r^T s_r to the x-part of K v,
// with s_r = w_r (P_r . v) (+ the weight of the A row it repeats) or, for a
// row of A, s_r = w_l - w_u: a function of the row's own dot (the matrix-free
// product of Section 3.2 is row-local).  So one pass over the rows forms the
// whole x-part, each stored entry read from HBM once and used twice: for the
// dot and, still in registers, for the scatter.
//
// One CU's LDS cannot hold both the gathered vector and the scatter target
// (2n float64 values at n = 20,000), so the columns are cut in two halves and
// each row range goes to a pair of blocks, block 2r + h owning half h: it
// keeps v's half and y's half in LDS, forms the half-h part of each row's dot
// and exchanges it with its partner through memory.  Both then hold the whole
// dot (added in the same order) and scatter their half of the row's entries
// into LDS with float64 atomics.  Each range's y is written to ypart (nrange
// x n) and the PCG update sums the ranges in order; the atomics' order
// varies, so products agree with the two-pass kernels to rounding, not
// bitwise.
//
// The exchange is per wave and needs no flag: wave w of either block takes
// the same rows (8 per tile, one per group of 8 lanes), stores each half dot
// in its slot of xch with a device-coherent store, and reads the partner's
// slot with a device-coherent load, which returns the sentinel (all bits
// set) until the partner's store has landed; the reader then puts the
// sentinel back.  Slots alternate with the launch parity, so a slot is
// rewritten only two launches later, after the reset.  Every wave pipelines
// its own tiles: in phase ph it scatters tile ph-2, issues the partner load
// of tile ph-1, the row bounds of tile ph+2 and the entries of tile ph+1,
// then forms tile ph's dots.  Loads are issued in the order they are waited
// for (the vector memory counter drains in issue order), so no wait holds a
// tile that is still in flight.  A wait for the partner is bounded: after
// f.spin_max polls the block sets the sticky abort flag and goes on; the
// product is then invalid and the host redoes the work with the two-pass
// kernels.

// Exchanges within a group of 8 lanes (a half row of the DPP unit), done by
// the VALU's data-parallel permutes rather than through the LDS crossbar:
// quad_perm moves values within 4 lanes, row_half_mirror maps lane i of
// 8 to lane 7 - i.
constexpr int kDppHalfMirror = 0x141;
constexpr int dpp_quad(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const i2v v = __builtin_bit_cast(i2v, x);
  i2v o;
  o.x = __builtin_amdgcn_update_dpp(0, v.x, CTRL, 0xf, 0xf, false);
  o.y = __builtin_amdgcn_update_dpp(0, v.y, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, o);
}
// Sum over the 8 lanes of the group, the same bits on every lane.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_f64<dpp_quad(1, 0, 3, 2)>(v);
  v += dpp_f64<dpp_quad(2, 3, 0, 1)>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  return v;
}
// Lane J's value of the group, on every lane of the group.
template <int J>
__device__ __forceinline__ double group8_bcast(double x) {
  const double y = dpp_f64<dpp_quad(J & 3, J & 3, J & 3, J & 3)>(x);   // lane J mod 4 of each quad
  const double z = dpp_f64<kDppHalfMirror>(y);                       // the other quad's
  const bool upper = (threadIdx.x & 4) != 0;
  return upper == (J >= 4) ? y : z;
}

// Row data of the epilogue, loaded ahead by role: in a tile's load phase
// lane 0 of the row's group fetches w_r (0 for a row of A) and lane 1 the
// row's rowinfo word: the index i_r of the row of A the row carries (its
// twin for a row of P, or itself), with bit 30 set when that row has a
// finite lower side and bit 29 a finite upper side, or -1 for none; after
// the tile's dot lanes 2..5 fetch that row of A's v_lo, v_up, d_lo, d_up.
constexpr int kRowLo = 1 << 30, kRowHi = 1 << 29, kRowIdx = kRowHi - 1;
__device__ __forceinline__ double fused_field(const RowArgs& a, int role, int i) {
  switch (role) {
    case 2: return a.vl[a.me + i];
    case 3: return a.vl[a.me + a.m + i];
    case 4: return a.dl[a.me + i];
    default: return a.dl[a.me + a.m + i];
  }
}

constexpr unsigned long long kFusedEmpty = ~0ull;   // an exchange slot not yet written

template <int VK, int PP>
__global__ __launch_bounds__(kChunkBlock) void k_fused(FusedArgs f, RowArgs ra) {
  using T = typename VT<VK>::T;
  using Acc = typename VT<VK>::Acc;
  constexpr int LPR = kFusedLpr;
  static_assert(LPR == 8, "the epilogue's row data is spread over eight lanes");
  constexpr int GW = 64 / LPR;                   // rows per wave tile
  constexpr int NW = kChunkBlock / 64;           // waves per block
  constexpr int SPAN = 2 * LPR * PP;             // entries per row per batch
  if (ra.done && *ra.done) return;
  if (ra.bump && blockIdx.x == 0 && threadIdx.x == 0) *ra.bump += 1;
  extern __shared__ __align__(16) double lds[];
  const int h = static_cast<int>(blockIdx.x & 1), r = static_cast<int>(blockIdx.x >> 1);
  const int c0 = h ? f.half : 0;
  const int cw = h ? f.ncols - f.half : f.half;
  double* vh = lds;                    // v_x[c0, c0 + cw)
  double* yh = lds + f.half;           // y_x[c0, c0 + cw)
  const int R0 = f.range[r], R1 = f.range[r + 1];
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  // this half's dots of the wave's rows, by tile mod 3 (kept here rather than
  // in registers from the dot to the scatter two phases later)
  double* owns = lds + 2 * f.half + wave * 3 * GW;
  const int g = (static_cast<int>(threadIdx.x) & 63) / LPR;   // group in the wave
  const int lane = threadIdx.x & (LPR - 1);
  // wave tile k holds rows R0 + (k NW + wave) GW + g
  const int nt = (R1 - R0 + NW * GW - 1) / (NW * GW);
  const int32_t* rp = f.rowptr + static_cast<int64_t>(h) * (f.nrows + 1);
  const T* val = static_cast<const T*>(f.val);
  const __amdgpu_buffer_rsrc_t rrp = rsrc(rp, 4u * static_cast<uint32_t>(f.nrows + 1));
  const __amdgpu_buffer_rsrc_t rcol = rsrc(f.col, 2u * static_cast<uint32_t>(f.nstored));
  const __amdgpu_buffer_rsrc_t rval = rsrc(val, static_cast<uint32_t>(sizeof(T)) * f.nstored);
  // exchange slots of this launch's parity: [half][row]
  double* xbase = f.xch + static_cast<int64_t>(f.epoch & 1) * 2 * f.nrows;
  double* xown = xbase + static_cast<int64_t>(h) * f.nrows;
  double* xother = xbase + static_cast<int64_t>(h ^ 1) * f.nrows;
  using LT = decltype(ldv(val, 0));

  {
    // stage v's half: every 16-byte load issued before the first LDS write,
    // so the block waits for one memory latency (c0 and the half are even)
    constexpr int SP = (kFusedHalfMax + 2 * kChunkBlock - 1) / (2 * kChunkBlock);
    const __amdgpu_buffer_rsrc_t rsv = rsrc(f.src + c0, 8u * static_cast<uint32_t>(cw));
    double2 st[SP];
#pragma unroll
    for (int k = 0; k < SP; ++k)
      st[k] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(
                                              rsv, 16u * (threadIdx.x + k * kChunkBlock), 0, 0));
    for (int i = threadIdx.x; i < cw; i += kChunkBlock) yh[i] = 0.0;
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int i2 = threadIdx.x + k * kChunkBlock;
      if (2 * i2 + 1 < cw) reinterpret_cast<double2*>(vh)[i2] = st[k];
    }
    if ((cw & 1) && threadIdx.x == 0) vh[cw - 1] = f.src[c0 + cw - 1];
  }

  struct Tile {
    uint32_t cc[PP];
    LT vx[PP], vy[PP];
    int beg, end;
    double fb;        // this lane's epilogue field (see fused_field)
    double xo;        // the partner's half dot, or the sentinel (every lane)
  };
  auto load_batch = [&](int base, int end, uint32_t* cc, LT* vx, LT* vy) {
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      const int q = base + 2 * (lane + k * LPR);
      const bool ok = q < end;
      cc[k] = __builtin_amdgcn_raw_buffer_load_b32(rcol, ok ? 2u * q : kOob, 0, 0);
      ldv2b(val, rval, ok ? static_cast<uint32_t>(sizeof(T)) * q : kOob, vx[k], vy[k]);
    }
  };
  auto row_of = [&](int k) { return R0 + (k * NW + wave) * GW + g; };
  auto row_ok = [&](int k) { return k >= 0 && k < nt && row_of(k) < R1; };
  // [rowptr[row], rowptr[row + 1]) of this group's row in tile k, else empty
  auto bounds = [&](int k, int& beg, int& end) {
    const i2v be = __builtin_bit_cast(
        i2v, __builtin_amdgcn_raw_buffer_load_b64(rrp, row_ok(k) ? 4u * row_of(k) : kOob, 0, 0));
    beg = be.x;
    end = be.y;
  };
  // lanes 0 and 1 fetch w_r and i_r, then every lane the entries of tile k
  auto load_tile = [&](Tile& tl, int k, int beg, int end) {
    tl.fb = 0.0;
    if (row_ok(k)) {
      const int row = row_of(k);
      if (lane == 0) tl.fb = row < ra.p_rows ? ra.w[row] : 0.0;
      if (lane == 1) tl.fb = static_cast<double>(f.rowinfo[row]);
    }
    tl.beg = beg;
    tl.end = end;
    load_batch(beg, end, tl.cc, tl.vx, tl.vy);
  };
  auto scatter_batch = [&](const uint32_t* cc, const LT* vx, const LT* vy, double s) {
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      // zero entries (the even-length padding, loads past the end) add nothing
      if (vx[k] != LT(0)) atomicAdd(&yh[cc[k] & 0xffffu], static_cast<double>(vx[k]) * s);
      if (vy[k] != LT(0)) atomicAdd(&yh[cc[k] >> 16], static_cast<double>(vy[k]) * s);
    }
  };

  double acc = 0.0;
  bool abandoned = __hip_atomic_load(f.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;

  // Epilogue of this group's row of tile k (lane 0; the row's data spread
  // over the group's lanes) and the scatter of its entries.
  auto scatter_tile = [&](Tile& tl, int k) {
    const bool valid = row_ok(k);
    double t = 0.0;
    if (valid) {     // every lane of the group, on the same slot
      const int row = row_of(k);
      unsigned long long bits = __builtin_bit_cast(unsigned long long, tl.xo);
      for (int spin = 0; bits == kFusedEmpty && !abandoned; ++spin) {
        // the partner has not stored this row's half dot yet
        if ((spin & 255) == 255 &&
            __hip_atomic_load(f.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
          abandoned = true;
        if (spin >= f.spin_max) {
          __hip_atomic_store(f.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          abandoned = true;
        }
        __builtin_amdgcn_s_sleep(2);
        bits = __builtin_bit_cast(unsigned long long,
                                  __hip_atomic_load(xother + row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      }
      const double o = bits == kFusedEmpty ? 0.0 : __builtin_bit_cast(double, bits);
      if (lane == 0)
        __hip_atomic_store(xother + row, __builtin_bit_cast(double, kFusedEmpty), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      const double own = owns[(k % 3) * GW + g];
      t = h == 0 ? own + o : o + own;     // half 0 first on both sides
    }
    const double w = group8_bcast<0>(tl.fb);
    const int info = static_cast<int>(group8_bcast<1>(tl.fb));
    const double vlo = group8_bcast<2>(tl.fb), vup = group8_bcast<3>(tl.fb);
    const double dlo = group8_bcast<4>(tl.fb), dup = group8_bcast<5>(tl.fb);
    if (!valid) return;
    const double uv = w * t;
    double wa = 0.0;
    if (info >= 0) {
      const int i = info & kRowIdx;
      const bool hl = (info & kRowLo) != 0, hu = (info & kRowHi) != 0;
      wa = (hl ? 2.0 * t / dlo + vlo : 0.0) - (hu ? -2.0 * t / dup + vup : 0.0);
      if (h == 0 && lane == 0) {
        // the lam-part of K v for this row of A, and its terms of p.q
        const double ylo = (hl ? t : 0.0) + dlo * vlo;
        const double yup = (hu ? -t : 0.0) + dup * vup;
        ra.yl[ra.me + i] = ylo;
        ra.yl[ra.me + ra.m + i] = yup;
        acc += vlo * ylo + vup * yup + t * wa;
      }
    }
    if (h == 0 && lane == 0) acc += t * uv;
    const double s = uv + wa;
    scatter_batch(tl.cc, tl.vx, tl.vy, s);
    for (int base = tl.beg + SPAN; base < tl.end; base += SPAN) {   // rows past one batch
      uint32_t c2[PP];
      LT x2[PP], y2[PP];
      load_batch(base, tl.end, c2, x2, y2);
      scatter_batch(c2, x2, y2, s);
    }
  };

  int nb = 0, ne = 0;    // bounds of the next tile to load, one phase ahead
  // one phase: scatter tile ph-2 (tsl), partner load of tile ph-1 (tw), bounds
  // of tile ph+2, entries of tile ph+1 (into tsl), dots of tile ph (td)
  auto phase = [&](int ph, Tile& td, Tile& tw, Tile& tsl) {
    if (ph >= 2) scatter_tile(tsl, ph - 2);
    tw.xo = 0.0;
    if (row_ok(ph - 1))
      tw.xo = __hip_atomic_load(xother + row_of(ph - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int cb = nb, ce = ne;
    bounds(ph + 2, nb, ne);
    load_tile(tsl, ph + 1, cb, ce);
    if (ph < nt) {
      Acc t = 0;
#pragma unroll
      for (int k = 0; k < PP; ++k) {
        t += static_cast<Acc>(td.vx[k]) * static_cast<Acc>(vh[td.cc[k] & 0xffffu]);
        t += static_cast<Acc>(td.vy[k]) * static_cast<Acc>(vh[td.cc[k] >> 16]);
      }
      for (int base = td.beg + SPAN; base < td.end; base += SPAN) {
        uint32_t c2[PP];
        LT x2[PP], y2[PP];
        load_batch(base, td.end, c2, x2, y2);
#pragma unroll
        for (int k = 0; k < PP; ++k) {
          t += static_cast<Acc>(x2[k]) * static_cast<Acc>(vh[c2[k] & 0xffffu]);
          t += static_cast<Acc>(y2[k]) * static_cast<Acc>(vh[c2[k] >> 16]);
        }
      }
      const double own = group8_sum(static_cast<double>(t));
      if (lane == 0) owns[(ph % 3) * GW + g] = own;
      if (lane == 0 && row_ok(ph))
        __hip_atomic_store(xown + row_of(ph), own, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // the row of A this row carries: lanes 2..5 fetch its fields
      const int info = static_cast<int>(group8_bcast<1>(td.fb));
      if (lane >= 2 && lane <= 5 && row_ok(ph) && info >= 0) td.fb = fused_field(ra, lane, info & kRowIdx);
    }
  };

  Tile A, B, C;
  {
    int b0, e0;
    bounds(0, b0, e0);
    bounds(1, nb, ne);
    load_tile(A, 0, b0, e0);
  }
  __syncthreads();    // v's half staged, y's half zeroed
  for (int ph = 0; ph < nt + 2; ph += 3) {
    phase(ph, A, C, B);
    if (ph + 1 < nt + 2) phase(ph + 1, B, A, C);
    if (ph + 2 < nt + 2) phase(ph + 2, C, B, A);
  }
  __syncthreads();    // every wave's scatters are in y's half

  for (int j = threadIdx.x; j < cw; j += kChunkBlock)
    f.ypart[static_cast<int64_t>(r) * f.ncols + c0 + j] = yh[j];
  // the terms of v_x . (K v)_x that are not row terms (equality rows,
  // diagonal): block (r, h) takes the r-th slice of half h
  if (ra.xdot) {
    const int j0 = c0 + static_cast<int>(static_cast<int64_t>(cw) * r / f.nrange);
    const int j1 = c0 + static_cast<int>(static_cast<int64_t>(cw) * (r + 1) / f.nrange);
    for (int j = j0 + threadIdx.x; j < j1; j += kChunkBlock) {
      const double vj = vh[j - c0];
      double e = 0.0;
      for (int i = 0; i < ra.me; ++i) e += ra.Cm[static_cast<int64_t>(i) * ra.n + j] * ra.we[i];
      acc += vj * e + ra.qdiag[j] * vj * vj;
    }
  }
  acc = block_sum_nt<kChunkBlock>(acc);
  if (threadIdx.x == 0) ra.part0[blockIdx.x] = acc;
}

// ------------------------------------------ tall-skinny dense reduction
// Block b reduces rows [b*chunk, (b+1)*chunk) of U (n x k, row-major) into
// part[b][0..k) and of C (me x n) into part[b][k..k+me).  Each wave owns a
// 64-column tile and every fourth row, so a wave reads 64 consecutive values
// of a row per step.
template <int VK>
__global__ __launch_bounds__(kBlock) void k_ts_reduce(TsArgs a) {
  using T = typename VT<VK>::T;
  using Acc = typename VT<VK>::Acc;
  if (a.done && *a.done) return;
  __shared__ double red[kBlock];
  const T* __restrict__ U = static_cast<const T*>(a.U);
  const int KW = a.k + a.me;
  const int j0 = blockIdx.x * a.chunk;
  const int j1 = min(a.n, j0 + a.chunk);
  double* out = a.part + static_cast<int64_t>(blockIdx.x) * KW;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if ((a.k & 1) == 0) {
    // even k: lane l owns columns 2l, 2l+1 of each 128-column tile, one
    // 16-byte (float64) load per row, so a wave reads 128 values of a row
    using LT = decltype(ldv(U, 0));
    __shared__ double red2[2 * kBlock];
    for (int c0 = 0; c0 < a.k; c0 += 128) {
      const int c = c0 + 2 * lane;
      Acc s0 = 0, s1 = 0;
      if (c < a.k) {
#pragma unroll 4
        for (int j = j0 + wv; j < j1; j += kBlock / 64) {
          LT ux, uy;
          ldv2(U, static_cast<int64_t>(j) * a.k + c, ux, uy);
          const Acc vj = static_cast<Acc>(a.v[j]);
          s0 += static_cast<Acc>(ux) * vj;
          s1 += static_cast<Acc>(uy) * vj;
        }
      }
      red2[2 * threadIdx.x] = static_cast<double>(s0);
      red2[2 * threadIdx.x + 1] = static_cast<double>(s1);
      __syncthreads();
      if (wv == 0 && c < a.k) {
        double t0 = red2[2 * lane], t1 = red2[2 * lane + 1];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) {
          t0 += red2[2 * (w * 64 + lane)];
          t1 += red2[2 * (w * 64 + lane) + 1];
        }
        out[c] = t0;
        out[c + 1] = t1;
      }
      __syncthreads();
    }
  } else
  for (int c0 = 0; c0 < a.k; c0 += 64) {
    const int c = c0 + lane;
    Acc acc = 0;
    if (c < a.k) {
      for (int j = j0 + wv; j < j1; j += kBlock / 64)
        acc += ldv(U, static_cast<int64_t>(j) * a.k + c) * static_cast<Acc>(a.v[j]);
    }
    red[threadIdx.x] = static_cast<double>(acc);
    __syncthreads();
    if (wv == 0 && c < a.k) {
      double s = red[lane];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) s += red[w * 64 + lane];
      out[c] = s;
    }
    __syncthreads();
  }
  for (int e = 0; e < a.me; ++e) {
    double acc = 0.0;
    for (int j = j0 + threadIdx.x; j < j1; j += kBlock)
      acc += a.Cm[static_cast<int64_t>(e) * a.n + j] * a.v[j];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[a.k + e] = acc;
  }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_ts_finish(TsFinishArgs a) {
  // Block l sums column l of the reduction's per-block partials (a.grid rows
  // of k + me): thread t takes rows t, t + kBlock, ..., then the block tree.
  if (a.done && *a.done) return;
  const int KW = a.k + a.me;
  const int l = blockIdx.x;
  double s = 0.0;
#pragma unroll 8
  for (int b = threadIdx.x; b < a.grid; b += kBlock) s += a.part[static_cast<int64_t>(b) * KW + l];
  s = block_sum(s);
  if (threadIdx.x != 0) return;
  if (l < a.k) {
    a.g[l] = a.wd[l] * s;
    return;
  }
  const int e = l - a.k;
  a.te[e] = s;
  // equality row e: its term of the product (TS_MATVEC) or of the residual
  // (TS_RESID); partout[e] is summed over e by the consumers
  if constexpr (MODE == TS_MATVEC) {
    const double ve = a.vl[e];
    a.we[e] = 2.0 * s / a.mu + ve;
    const double ye = s + a.mu * ve;
    a.yl[e] = ye;
    a.partout[e] = ve * ye;
  } else if constexpr (MODE == TS_RESID) {
    const double re = s - a.b[e] + a.mu * a.lam[e];
    a.res[a.n + e] = re;
    a.we[e] = -a.lam[e];
    a.partout[e] = re * re;
  }
}

// ------------------------------------------------------ IPM step kernels
// Right-hand side rows of the lam-part and the D blocks (eq. (8)/(9)):
//   D = (mu, s_lA/lam_lA, s_uA/lam_uA),  r2 = (-r_e, -r_lA - r_c1/lam_lA, -r_uA - r_c2/lam_uA)
// plus the per-row weights of 2 B^T D^-1 r2 (wA) and of diag(2 B^T D^-1 B) (jw).
__global__ __launch_bounds__(kBlock) void k_rhs_lam(VecArgs a) {
  const int n = a.n, m = a.m, me = a.me;
  const ResOff o(n, m, me);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < me + m; i += gridDim.x * kBlock) {
    if (i < me) {
      const double r2 = -a.res[o.re + i];
      a.rhs[n + i] = r2;
      a.jdiag[n + i] = a.mu;
      a.dl[i] = a.mu;
      a.we[i] = 2.0 * r2 / a.mu;
      continue;
    }
    const int r = i - me;
    const bool hl = has_lo(a.lA[r]), hu = has_hi(a.uA[r]);
    const double ll = a.lam[me + r], lu = a.lam[me + m + r];
    const double dL = hl ? a.s[r] / ll : 1.0;
    const double dU = hu ? a.s[m + r] / lu : 1.0;
    const double r2L = hl ? -a.res[o.rlA + r] - a.res[o.rc1 + r] / ll : 0.0;
    const double r2U = hu ? -a.res[o.ruA + r] - a.res[o.rc2 + r] / lu : 0.0;
    a.rhs[n + me + r] = r2L;
    a.rhs[n + me + m + r] = r2U;
    a.jdiag[n + me + r] = dL;
    a.jdiag[n + me + m + r] = dU;
    a.dl[me + r] = dL;
    a.dl[me + m + r] = dU;
    a.wA[r] = (hl ? 2.0 * r2L / dL : 0.0) - (hu ? 2.0 * r2U / dU : 0.0);
    a.jw[r] = (hl ? 2.0 / dL : 0.0) + (hu ? 2.0 / dU : 0.0);
  }
}

// Variable-bound part of the recovery (complementarity rows of eq. (7)) and
// of the ratio test (eq. (10)).
__global__ __launch_bounds__(kBlock) void k_recover_x(VecArgs a) {
  const int n = a.n, m = a.m, me = a.me;
  const ResOff o(n, m, me);
  double ms = INFINITY, ml = INFINITY;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
    const bool hl = has_lo(a.lx[j]), hu = has_hi(a.ux[j]);
    const double dxj = a.dx[j];
    double dsl = 0.0, dsu = 0.0, dll = 0.0, dlu = 0.0;
    if (hl) {
      const double slx = a.s[2 * m + j], llx = a.lam[me + 2 * m + j];
      dsl = dxj + a.res[o.rlx + j];
      dll = -(a.res[o.rc3 + j] + llx * dsl) / slx;
      if (dsl < 0.0) ms = fmin(ms, -slx / dsl);
      if (dll < 0.0) ml = fmin(ml, -llx / dll);
    }
    if (hu) {
      const double sux = a.s[2 * m + n + j], lux = a.lam[me + 2 * m + n + j];
      dsu = -dxj + a.res[o.rux + j];
      dlu = -(a.res[o.rc4 + j] + lux * dsu) / sux;
      if (dsu < 0.0) ms = fmin(ms, -sux / dsu);
      if (dlu < 0.0) ml = fmin(ml, -lux / dlu);
    }
    a.ds[2 * m + j] = dsl;
    a.ds[2 * m + n + j] = dsu;
    a.dlam_w[me + 2 * m + j] = dll;
    a.dlam_w[me + 2 * m + n + j] = dlu;
  }
  ms = block_min(ms);
  ml = block_min(ml);
  if (threadIdx.x == 0) {
    a.part[P_MIN_S_X * kGridMax + blockIdx.x] = ms;
    a.part[P_MIN_L_X * kGridMax + blockIdx.x] = ml;
  }
}

// alpha = min(1, gamma * min ratio); an empty set gives 1 (eq. (10)).
__global__ __launch_bounds__(kBlock) void k_finish_ratio(VecArgs a, int g_r, int g_x) {
  const double* P = a.part;
  const double ms = fmin(min_bcast(P + P_MIN_S_R * kGridMax, g_r), min_bcast(P + P_MIN_S_X * kGridMax, g_x));
  const double ml = fmin(min_bcast(P + P_MIN_L_R * kGridMax, g_r), min_bcast(P + P_MIN_L_X * kGridMax, g_x));
  if (threadIdx.x == 0) {
    a.sc[S_ALPHA_X] = fmin(1.0, a.gamma * ms);
    a.sc[S_ALPHA_L] = fmin(1.0, a.gamma * ml);
  }
}

// Stacked residual norm and the three infeasibilities of Section 5.2.
__global__ __launch_bounds__(kBlock) void k_finish_norms(VecArgs a, int g_r, int g_x) {
  const double* P = a.part;
  const double pr = sum_bcast(P + P_NR_PRIMAL * kGridMax, g_r) + sum_bcast(P + P_NX_PRIMAL * kGridMax, g_x);
  const double du = sum_bcast(P + P_NX_DUAL * kGridMax, g_x);
  const double co = sum_bcast(P + P_NR_COMPL * kGridMax, g_r) + sum_bcast(P + P_NX_COMPL * kGridMax, g_x);
  double re = 0.0;
  for (int e = 0; e < a.me; ++e) re += P[P_NTS_RE * kGridMax + e];
  if (threadIdx.x == 0) {
    a.sc[S_NORM] = sqrt(pr + du + co + re);
    a.sc[S_PRIMAL] = sqrt(pr);
    a.sc[S_DUAL] = sqrt(du);
    a.sc[S_COMPL] = sqrt(co);
  }
}

__global__ __launch_bounds__(kBlock) void k_finish_sum(const double* part, int count, double* out) {
  const double s = sum_bcast(part, count);
  if (threadIdx.x == 0) *out = s;
}

// x += ax dx, s += ax ds, lam += al dlam over present entries (Algorithm 1).
__global__ __launch_bounds__(kBlock) void k_update(VecArgs a, const double* dx, const double* dlam,
                                                  const double* ds, const double* alpha_dev,
                                                  double ax, double al) {
  const int n = a.n, m = a.m, me = a.me;
  if (alpha_dev) {
    ax = alpha_dev[0];
    al = alpha_dev[1];
  }
  const int total = me + 2 * m + 2 * n;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    if (i < n) a.x[i] += ax * dx[i];
    bool present;
    if (i < me) {
      a.lam[i] += al * dlam[i];
    } else {
      const int q = i - me;  // index into the s layout
      if (q < m) present = has_lo(a.lA[q]);
      else if (q < 2 * m) present = has_hi(a.uA[q - m]);
      else if (q < 2 * m + n) present = has_lo(a.lx[q - 2 * m]);
      else present = has_hi(a.ux[q - 2 * m - n]);
      if (present) {
        a.lam[i] += al * dlam[i];
        a.s[q] += ax * ds[q];
      }
    }
  }
}

// Default starting point, variable part (the row slacks follow in R_INIT).
__global__ __launch_bounds__(kBlock) void k_init_x(VecArgs a) {
  const int n = a.n, m = a.m, me = a.me;
  const int total = n > me ? n : me;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < total; j += gridDim.x * kBlock) {
    if (j < me) a.lam[j] = 0.0;
    if (j >= n) continue;
    const double l = a.lx[j], u = a.ux[j];
    const bool hl = has_lo(l), hu = has_hi(u);
    double x = 0.0;
    if (hl && hu) x = 0.5 * (l + u);
    else if (hl) x = l + 1.0;
    else if (hu) x = u - 1.0;
    a.x[j] = x;
    a.s[2 * m + j] = hl ? x - l : 0.0;
    a.s[2 * m + n + j] = hu ? u - x : 0.0;
    a.lam[me + 2 * m + j] = hl ? 1.0 : 0.0;
    a.lam[me + 2 * m + n + j] = hu ? 1.0 : 0.0;
  }
}

// Validates a caller iterate: counts present entries that are not finite and
// positive, and zeroes the entries of absent sides.
__global__ __launch_bounds__(kBlock) void k_check_state(VecArgs a) {
  const int n = a.n, m = a.m, me = a.me;
  const int total = me + 2 * m + 2 * n;
  double bad = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    if (i < n && !isfinite(a.x[i])) bad += 1.0;
    if (i < me) {
      if (!isfinite(a.lam[i])) bad += 1.0;
      continue;
    }
    const int q = i - me;
    bool present;
    if (q < m) present = has_lo(a.lA[q]);
    else if (q < 2 * m) present = has_hi(a.uA[q - m]);
    else if (q < 2 * m + n) present = has_lo(a.lx[q - 2 * m]);
    else present = has_hi(a.ux[q - 2 * m - n]);
    if (present) {
      const double l = a.lam[i], s = a.s[q];
      if (!(isfinite(l) && l > 0.0 && isfinite(s) && s > 0.0)) bad += 1.0;
    } else {
      a.lam[i] = 0.0;
      a.s[q] = 0.0;
    }
  }
  bad = block_sum(bad);
  if (threadIdx.x == 0) a.part[P_CHK * kGridMax + blockIdx.x] = bad;
}

// ------------------------------------------------------------ PCG kernels
// Textbook Jacobi PCG on eq. (9) (Sections 3.1, 5.1): x0 = 0, z = r / diag,
// stop when ||r||_2 <= tol ||rhs||_2 or at maxit.  Scalars are never stored by
// one block for the others: every block re-sums the partials it needs, so the
// only cross-block state is the partial arrays and the flags.  rz partials
// alternate between two regions by iteration parity.
__global__ __launch_bounds__(kBlock) void k_cg_init(CgArgs a) {
  double rz = 0.0, rr = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.N; i += gridDim.x * kBlock) {
    const double r = a.rhs[i];
    const double z = r / a.jdiag[i];
    a.x[i] = 0.0;
    a.r[i] = r;
    a.z[i] = z;
    a.p[i] = z;
    rz += r * z;
    rr += r * r;
  }
  rz = block_sum(rz);
  rr = block_sum(rr);
  if (threadIdx.x == 0) {
    a.part[P_RZ0 * kGridMax + blockIdx.x] = rz;
    a.part[P_RR0 * kGridMax + blockIdx.x] = rr;
    if (blockIdx.x == 0) {
      a.fl[F_DONE] = 0;
      a.fl[F_CNT] = -1;
      a.fl[F_STATUS] = 0;
      a.fl[F_ITERS] = 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_init_finish(CgArgs a) {
  const double rr0 = sum_bcast(a.part + P_RR0 * kGridMax, a.g_vec);
  if (threadIdx.x == 0) {
    a.sc[S_RHSNORM] = sqrt(rr0);
    if (!(rr0 > 0.0)) {
      a.fl[F_DONE] = 1;
      a.fl[F_STATUS] = (rr0 == 0.0) ? 1 : QP_ERR_NUMERIC_CODE;
    }
  }
}

// The vector loads of a thread's first element are issued before the
// partial sums are read, so the two memory latencies overlap.
__global__ __launch_bounds__(kBlock) void k_cg_update(CgArgs a) {
  const int stride = gridDim.x * kBlock;
  int i = blockIdx.x * kBlock + threadIdx.x;
  double xi = 0.0, pi = 0.0, ri = 0.0, qi = 0.0, di = 1.0;
  if (i < a.N) {
    xi = a.x[i];
    pi = a.p[i];
    ri = a.r[i];
    di = a.jdiag[i];
    qi = a.q[i];
  }
  if (a.fl[F_DONE]) return;
  const int k = a.fl[F_CNT];
  const double* P = a.part;
  double pqr, pqx, rz;
  sum3_bcast(P + P_DOT_R * kGridMax, a.g_r, P + P_DOT_X * kGridMax, a.g_x,
             P + ((k & 1) ? P_RZ1 : P_RZ0) * kGridMax, a.g_vec, pqr, pqx, rz);
  double pq = pqr + pqx;
  if (a.has_ts)
    for (int e = 0; e < a.me; ++e) pq += P[P_DOT_TS * kGridMax + e];
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.fl[F_STATUS] = (isfinite(pq) && isfinite(rz)) ? QP_ERR_NOT_SPD_CODE : QP_ERR_NUMERIC_CODE;
      a.fl[F_ITERS] = k;
      a.fl[F_DONE] = 1;
    }
    return;
  }
  const double alpha = rz / pq;
  if (a.coef && blockIdx.x == 0 && threadIdx.x == 0) a.coef[2 * k] = alpha;
  double rzn = 0.0, rr = 0.0;
  for (; i < a.N; i += stride) {
    a.x[i] = xi + alpha * pi;
    const double r = ri - alpha * qi;
    const double z = r / di;
    a.r[i] = r;
    a.z[i] = z;
    rzn += r * z;
    rr += r * r;
    const int j = i + stride;
    if (j < a.N) {
      xi = a.x[j];
      pi = a.p[j];
      ri = a.r[j];
      di = a.jdiag[j];
      qi = a.q[j];
    }
  }
  rzn = block_sum(rzn);
  rr = block_sum(rr);
  if (threadIdx.x == 0) {
    a.part[(((k + 1) & 1) ? P_RZ1 : P_RZ0) * kGridMax + blockIdx.x] = rzn;
    a.part[P_RR * kGridMax + blockIdx.x] = rr;
  }
}

// k_cg_update when the x-part of q comes from per-chunk (or per-range)
// partials: each wave takes 16 entries of the x-part, a quarter of the wave
// per chunk group, so every lane has at most ceil(nchunk / 4) loads to wait
// for, all in flight together, and the x-part is spread over the whole grid
// instead of the first blocks.  The groups' sums meet by two lane exchanges,
// in the order sum_partials uses.  The rest of K v (the lam-part) is read
// from q, 64 entries per wave.  Every wave's first task is loaded before the
// scalar sums are read, as in k_cg_update.
struct UpdTask {
  int i;
  bool own;          // this lane updates entry i
  double xi, pi, ri, di, y;
};

__device__ __forceinline__ UpdTask upd_load(const CgArgs& a, int t, int xw, int lane) {
  UpdTask u;
  u.xi = u.pi = u.ri = 0.0;
  u.di = 1.0;
  u.y = 0.0;
  if (t < xw) {
    u.i = t * 16 + (lane & 15);
    u.own = lane < 16 && u.i < a.n;
    if (u.i < a.n) {
      const int g = partial_group(a.nchunk);
      const int c0 = (lane >> 4) * g, c1 = min(a.nchunk, c0 + g);
      const double* p = a.qpart + u.i;
      const int64_t st = a.n;
      for (int cb = c0; cb < c1; cb += 32) {
        double v[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) v[c] = cb + c < c1 ? p[(cb + c) * st] : 0.0;
#pragma unroll
        for (int c = 0; c < 32; ++c)
          if (cb + c < c1) u.y += v[c];
      }
    }
  } else {
    u.i = a.n + (t - xw) * 64 + lane;
    u.own = u.i < a.N;
    if (u.own) u.y = a.q[u.i];
  }
  if (u.own) {
    u.xi = a.x[u.i];
    u.pi = a.p[u.i];
    u.ri = a.r[u.i];
    u.di = a.jdiag[u.i];
  }
  return u;
}

__global__ __launch_bounds__(kBlock) void k_cg_update_split(CgArgs a) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (kBlock / 64);
  const int xw = (a.n + 15) >> 4;
  const int tasks = xw + (a.N - a.n + 63) / 64;
  int t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  UpdTask u = upd_load(a, t, xw, lane);
  if (a.fl[F_DONE]) return;
  const int k = a.fl[F_CNT];
  const double* P = a.part;
  double pqr, pqx, rz;
  sum3_bcast(P + P_DOT_R * kGridMax, a.g_r, P + P_DOT_X * kGridMax, a.g_x,
             P + ((k & 1) ? P_RZ1 : P_RZ0) * kGridMax, a.g_vec, pqr, pqx, rz);
  double pq = pqr + pqx;
  if (a.has_ts)
    for (int e = 0; e < a.me; ++e) pq += P[P_DOT_TS * kGridMax + e];
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.fl[F_STATUS] = (isfinite(pq) && isfinite(rz)) ? QP_ERR_NOT_SPD_CODE : QP_ERR_NUMERIC_CODE;
      a.fl[F_ITERS] = k;
      a.fl[F_DONE] = 1;
    }
    return;
  }
  const double alpha = rz / pq;
  if (a.coef && blockIdx.x == 0 && threadIdx.x == 0) a.coef[2 * k] = alpha;
  double rzn = 0.0, rr = 0.0;
  for (; t < tasks; t += nw) {
    double qi = u.y;
    if (t < xw) {
      const double y01 = qi + __shfl_xor(qi, 16, 64);
      qi = y01 + __shfl_xor(y01, 32, 64);
      if (u.own) {
        for (int e = 0; e < a.me; ++e) qi += a.Cm[static_cast<int64_t>(e) * a.n + u.i] * a.we[e];
        qi += a.qdiag[u.i] * u.pi;
      }
    }
    if (u.own) {
      a.x[u.i] = u.xi + alpha * u.pi;
      const double r = u.ri - alpha * qi;
      const double z = r / u.di;
      a.r[u.i] = r;
      a.z[u.i] = z;
      rzn += r * z;
      rr += r * r;
    }
    if (t + nw < tasks) u = upd_load(a, t + nw, xw, lane);
  }
  rzn = block_sum(rzn);
  rr = block_sum(rr);
  if (threadIdx.x == 0) {
    a.part[(((k + 1) & 1) ? P_RZ1 : P_RZ0) * kGridMax + blockIdx.x] = rzn;
    a.part[P_RR * kGridMax + blockIdx.x] = rr;
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_pupdate(CgArgs a) {
  const int stride = gridDim.x * kBlock;
  int i = blockIdx.x * kBlock + threadIdx.x;
  double zi = 0.0, pi = 0.0;
  if (i < a.N) {
    zi = a.z[i];
    pi = a.p[i];
  }
  if (a.fl[F_DONE]) return;
  const int k = a.fl[F_CNT];
  const double* P = a.part;
  double rz_old, rz_new, rr;
  sum3_bcast(P + ((k & 1) ? P_RZ1 : P_RZ0) * kGridMax, a.g_vec,
             P + (((k + 1) & 1) ? P_RZ1 : P_RZ0) * kGridMax, a.g_vec, P + P_RR * kGridMax, a.g_vec,
             rz_old, rz_new, rr);
  const bool conv = sqrt(rr) <= a.tol * a.sc[S_RHSNORM];
  if (conv || k + 1 >= a.maxit) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.fl[F_ITERS] = k + 1;
      a.fl[F_STATUS] = conv ? 1 : 2;
      a.fl[F_DONE] = 1;
    }
    return;
  }
  const double beta = rz_new / rz_old;
  if (a.coef && blockIdx.x == 0 && threadIdx.x == 0) a.coef[2 * k + 1] = beta;
  for (; i < a.N; i += stride) {
    a.p[i] = zi + beta * pi;
    const int j = i + stride;
    if (j < a.N) {
      zi = a.z[j];
      pi = a.p[j];
    }
  }
}

// Residual replacement for the reduced-precision operator (the reliable-update
// form of van der Vorst and Ye, 2000): r = rhs - K x with the float64 operator,
// z = r / diag, and the search direction p is kept, so the Krylov process goes
// on; the next alpha uses the replaced r . z.  On a resume (the recurrence
// residual met the tolerance but the float64 one did not) the replaced residual
// is unrelated to p, so the search restarts from p = z.
__global__ __launch_bounds__(kBlock) void k_cg_restart(CgArgs a, const double* kx, int resume) {
  if (!resume && a.fl[F_DONE]) return;
  const int k = a.fl[F_CNT] + 1;  // the iteration about to run
  double rz = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.N; i += gridDim.x * kBlock) {
    const double r = a.rhs[i] - kx[i];
    const double z = r / a.jdiag[i];
    a.r[i] = r;
    a.z[i] = z;
    if (resume) a.p[i] = z;
    rz += r * z;
  }
  rz = block_sum(rz);
  if (threadIdx.x == 0) a.part[((k & 1) ? P_RZ1 : P_RZ0) * kGridMax + blockIdx.x] = rz;
}

// Re-arms the iteration after a resume (the stop flag was set on the
// recurrence residual, but the float64 residual is not yet small enough).
__global__ void k_cg_rearm(int* fl) {
  if (threadIdx.x == 0) {
    fl[F_DONE] = 0;
    fl[F_STATUS] = 0;
  }
}

// Mehrotra predictor-corrector rule (an alternative to Algorithm 1's mu
// update): the complementarity sums over the inequality pairs, in the slack
// layout q = [lA (m) | uA (m) | lx (n) | ux (n)] with lam[me + q] the
// multiplier of slack q.  Absent sides hold zeros in lam, s and the
// direction, so they add nothing to the sums; they are left out of the count.
__global__ __launch_bounds__(kBlock) void k_compl(VecArgs a, const double* dlam, const double* ds,
                                                 double* part0, double* part1, double* part2) {
  const int n = a.n, m = a.m, me = a.me;
  const int ns = 2 * (m + n);
  const double ax = dlam ? a.sc[S_ALPHA_X] : 0.0, al = dlam ? a.sc[S_ALPHA_L] : 0.0;
  double c0 = 0.0, c1 = 0.0, cnt = 0.0;
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < ns; q += gridDim.x * kBlock) {
    const double l = a.lam[me + q], sq = a.s[q];
    c0 += l * sq;
    if (dlam) c1 += (l + al * dlam[me + q]) * (sq + ax * ds[q]);
    bool present;
    if (q < m) present = has_lo(a.lA[q]);
    else if (q < 2 * m) present = has_hi(a.uA[q - m]);
    else if (q < 2 * m + n) present = has_lo(a.lx[q - 2 * m]);
    else present = has_hi(a.ux[q - 2 * m - n]);
    cnt += present ? 1.0 : 0.0;
  }
  c0 = block_sum(c0);
  c1 = block_sum(c1);
  cnt = block_sum(cnt);
  if (threadIdx.x == 0) {
    part0[blockIdx.x] = c0;
    part1[blockIdx.x] = c1;
    part2[blockIdx.x] = cnt;
  }
}

// The corrector's right side: each complementarity residual (r_c1..r_c4,
// consecutive in the stack, in the slack layout) gains the predictor's
// dlam * ds, so the complementarity rows read lam ds + s dlam = tau - lam s -
// dlam^a ds^a.
__global__ __launch_bounds__(kBlock) void k_second_order(VecArgs a, double* res, const double* dlam,
                                                        const double* ds) {
  const ResOff o(a.n, a.m, a.me);
  const int ns = 2 * (a.m + a.n);
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < ns; q += gridDim.x * kBlock)
    res[o.rc1 + q] += dlam[a.me + q] * ds[q];
}

// Squared distance partials (true residual ||rhs - K x||^2).
__global__ __launch_bounds__(kBlock) void k_sqdiff(const double* a, const double* b, int64_t n,
                                                  double* part) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double d = a[i] - b[i];
    acc += d * d;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Ratio test of eq. (10) for a caller-given direction (iterate layouts).
__global__ __launch_bounds__(kBlock) void k_ratio_given(VecArgs a, const double* dlam, const double* ds) {
  const int n = a.n, m = a.m, me = a.me;
  double ms = INFINITY, ml = INFINITY;
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < 2 * m + 2 * n; q += gridDim.x * kBlock) {
    bool present;
    if (q < m) present = has_lo(a.lA[q]);
    else if (q < 2 * m) present = has_hi(a.uA[q - m]);
    else if (q < 2 * m + n) present = has_lo(a.lx[q - 2 * m]);
    else present = has_hi(a.ux[q - 2 * m - n]);
    if (!present) continue;
    const double dsq = ds[q], dlq = dlam[me + q];
    if (dsq < 0.0) ms = fmin(ms, -a.s[q] / dsq);
    if (dlq < 0.0) ml = fmin(ml, -a.lam[me + q] / dlq);
  }
  ms = block_min(ms);
  ml = block_min(ml);
  if (threadIdx.x == 0) {
    a.part[P_MIN_S_X * kGridMax + blockIdx.x] = ms;
    a.part[P_MIN_L_X * kGridMax + blockIdx.x] = ml;
  }
}

// ------------------------------------------------------------- backward
__global__ __launch_bounds__(kBlock) void k_grad_out(int n, int m, int me, const double* u,
                                                    const double* lA, const double* uA,
                                                    double* gc, double* glA, double* guA,
                                                    double* gb) {
  const int total = n > m ? n : m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    if (gc && i < n) gc[i] = -u[i];
    if (i < m) {
      if (glA) glA[i] = has_lo(lA[i]) ? -u[n + me + i] : 0.0;
      if (guA) guA[i] = has_hi(uA[i]) ? u[n + me + m + i] : 0.0;
    }
    if (gb && i < me) gb[i] = -u[n + i];
  }
}

__global__ __launch_bounds__(kBlock) void k_copy(const double* src, double* dst, int64_t n, double scale) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    dst[i] = scale * src[i];
}

__global__ __launch_bounds__(kBlock) void k_fill(double* dst, int64_t n, double v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    dst[i] = v;
}

// ------------------------------------------------------------- launchers
static inline int grid_for(int64_t items, int per_block) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > kGridMax) g = kGridMax;
  return static_cast<int>(g);
}

template <int MODE, int VK>
static hipError_t rowpass_lpr(int lpr, const RowArgs& a, int grid, hipStream_t st,
                              const KEvents* ev) {
  switch (lpr) {
    case 4: return launch_ev(ev, k_rowpass<MODE, VK, 4>, dim3(grid), dim3(kBlock), 0, st, a);
    case 8: return launch_ev(ev, k_rowpass<MODE, VK, 8>, dim3(grid), dim3(kBlock), 0, st, a);
    case 16: return launch_ev(ev, k_rowpass<MODE, VK, 16>, dim3(grid), dim3(kBlock), 0, st, a);
    case 32: return launch_ev(ev, k_rowpass<MODE, VK, 32>, dim3(grid), dim3(kBlock), 0, st, a);
    default: return launch_ev(ev, k_rowpass<MODE, VK, 64>, dim3(grid), dim3(kBlock), 0, st, a);
  }
  return hipGetLastError();
}

template <int MODE, int VK>
static hipError_t colpass_lpr(int lpr, const ColArgs& a, int grid, hipStream_t st,
                              const KEvents* ev) {
  switch (lpr) {
    case 4: return launch_ev(ev, k_colpass<MODE, VK, 4>, dim3(grid), dim3(kBlock), 0, st, a);
    case 8: return launch_ev(ev, k_colpass<MODE, VK, 8>, dim3(grid), dim3(kBlock), 0, st, a);
    case 16: return launch_ev(ev, k_colpass<MODE, VK, 16>, dim3(grid), dim3(kBlock), 0, st, a);
    case 32: return launch_ev(ev, k_colpass<MODE, VK, 32>, dim3(grid), dim3(kBlock), 0, st, a);
    default: return launch_ev(ev, k_colpass<MODE, VK, 64>, dim3(grid), dim3(kBlock), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_rowpass(int mode, int vk, int lpr, const RowArgs& a, int grid, hipStream_t st,
                          const KEvents* ev) {
  if (mode == R_MATVEC) {
    if (vk == VK_F32) return rowpass_lpr<R_MATVEC, VK_F32>(lpr, a, grid, st, ev);
    if (vk == VK_BF16) return rowpass_lpr<R_MATVEC, VK_BF16>(lpr, a, grid, st, ev);
    if (vk == VK_F32X) return rowpass_lpr<R_MATVEC, VK_F32X>(lpr, a, grid, st, ev);
    if (vk == VK_BF16X) return rowpass_lpr<R_MATVEC, VK_BF16X>(lpr, a, grid, st, ev);
    return rowpass_lpr<R_MATVEC, VK_F64>(lpr, a, grid, st, ev);
  }
  switch (mode) {
    case R_RESID: return rowpass_lpr<R_RESID, VK_F64>(lpr, a, grid, st, ev);
    case R_RECOVER: return rowpass_lpr<R_RECOVER, VK_F64>(lpr, a, grid, st, ev);
    case R_GRADW: return rowpass_lpr<R_GRADW, VK_F64>(lpr, a, grid, st, ev);
    case R_PU: return rowpass_lpr<R_PU, VK_F64>(lpr, a, grid, st, ev);
    case R_INIT: return rowpass_lpr<R_INIT, VK_F64>(lpr, a, grid, st, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_colpass(int mode, int vk, int lpr, const ColArgs& a, int grid, hipStream_t st,
                          const KEvents* ev) {
  if (mode == X_MATVEC) {
    if (vk == VK_F32) return colpass_lpr<X_MATVEC, VK_F32>(lpr, a, grid, st, ev);
    if (vk == VK_BF16) return colpass_lpr<X_MATVEC, VK_BF16>(lpr, a, grid, st, ev);
    if (vk == VK_F32X) return colpass_lpr<X_MATVEC, VK_F32X>(lpr, a, grid, st, ev);
    if (vk == VK_BF16X) return colpass_lpr<X_MATVEC, VK_BF16X>(lpr, a, grid, st, ev);
    return colpass_lpr<X_MATVEC, VK_F64>(lpr, a, grid, st, ev);
  }
  switch (mode) {
    case X_RESID: return colpass_lpr<X_RESID, VK_F64>(lpr, a, grid, st, ev);
    case X_RHS: return colpass_lpr<X_RHS, VK_F64>(lpr, a, grid, st, ev);
    case X_DIAGH: return colpass_lpr<X_DIAGH, VK_F64>(lpr, a, grid, st, ev);
    case X_CEFF: return colpass_lpr<X_CEFF, VK_F64>(lpr, a, grid, st, ev);
    case X_OBJ: return colpass_lpr<X_OBJ, VK_F64>(lpr, a, grid, st, ev);
    default: return hipErrorInvalidValue;
  }
}

template <int EPI, int VK, int KV>
static hipError_t chunked_lpr_kv(int lpr, const ChunkArgs& c, const RowArgs& ra, const ColArgs& ca,
                                 int nwork, hipStream_t st, const KEvents* ev) {
  const size_t lds = sizeof(double) * c.chunk_cols;
  const dim3 g(nwork), bl(kChunkBlock);
  switch (lpr) {
    case 4: return launch_ev(ev, k_chunked<EPI, VK, 4, KV>, g, bl, lds, st, c, ra, ca);
    case 8: return launch_ev(ev, k_chunked<EPI, VK, 8, KV>, g, bl, lds, st, c, ra, ca);
    case 16: return launch_ev(ev, k_chunked<EPI, VK, 16, KV>, g, bl, lds, st, c, ra, ca);
    case 32: return launch_ev(ev, k_chunked<EPI, VK, 32, KV>, g, bl, lds, st, c, ra, ca);
    default: return launch_ev(ev, k_chunked<EPI, VK, 64, KV>, g, bl, lds, st, c, ra, ca);
  }
}

// float64 row-side and multi-chunk passes come in both staging variants; the
// others use kKvDefault.
template <int EPI, int VK>
constexpr bool kv_all() { return VK == VK_F64 && EPI != CE_COL; }

template <int EPI, int VK>
static hipError_t chunked_lpr(int lpr, const ChunkArgs& c, const RowArgs& ra, const ColArgs& ca,
                              int nwork, hipStream_t st, const KEvents* ev) {
  if constexpr (kv_all<EPI, VK>()) {
    if (c.kv == 0) return chunked_lpr_kv<EPI, VK, 0>(lpr, c, ra, ca, nwork, st, ev);
    return chunked_lpr_kv<EPI, VK, 1>(lpr, c, ra, ca, nwork, st, ev);
  }
  return chunked_lpr_kv<EPI, VK, kKvDefault>(lpr, c, ra, ca, nwork, st, ev);
}

template <int EPI>
static hipError_t chunked_vk(int vk, int lpr, const ChunkArgs& c, const RowArgs& ra,
                             const ColArgs& ca, int nwork, hipStream_t st, const KEvents* ev) {
  if (vk == VK_F32) return chunked_lpr<EPI, VK_F32>(lpr, c, ra, ca, nwork, st, ev);
  if (vk == VK_BF16) return chunked_lpr<EPI, VK_BF16>(lpr, c, ra, ca, nwork, st, ev);
  if (vk == VK_F32X) return chunked_lpr<EPI, VK_F32X>(lpr, c, ra, ca, nwork, st, ev);
  if (vk == VK_BF16X) return chunked_lpr<EPI, VK_BF16X>(lpr, c, ra, ca, nwork, st, ev);
  return chunked_lpr<EPI, VK_F64>(lpr, c, ra, ca, nwork, st, ev);
}

hipError_t launch_chunked(int epi, int vk, int lpr, const ChunkArgs& c, const RowArgs& ra,
                          const ColArgs& ca, int nwork, hipStream_t st, const KEvents* ev) {
  if (epi == CE_ROW) return chunked_vk<CE_ROW>(vk, lpr, c, ra, ca, nwork, st, ev);
  if (epi == CE_COL) return chunked_vk<CE_COL>(vk, lpr, c, ra, ca, nwork, st, ev);
  return chunked_vk<CE_PARTIAL>(vk, lpr, c, ra, ca, nwork, st, ev);
}

template <int EPI, int VK, int KV>
static hipError_t set_attr_kv() {
  const int lds = sizeof(double) * kChunkCols;
  hipError_t e = hipSuccess;
  auto one = [&](const void* f) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  };
  one(reinterpret_cast<const void*>(&k_chunked<EPI, VK, 4, KV>));
  one(reinterpret_cast<const void*>(&k_chunked<EPI, VK, 8, KV>));
  one(reinterpret_cast<const void*>(&k_chunked<EPI, VK, 16, KV>));
  one(reinterpret_cast<const void*>(&k_chunked<EPI, VK, 32, KV>));
  one(reinterpret_cast<const void*>(&k_chunked<EPI, VK, 64, KV>));
  return e;
}

template <int EPI, int VK>
static hipError_t set_attr_lpr() {
  if constexpr (kv_all<EPI, VK>()) {
    hipError_t e = set_attr_kv<EPI, VK, 0>();
    if (e == hipSuccess) e = set_attr_kv<EPI, VK, 1>();
    return e;
  }
  return set_attr_kv<EPI, VK, kKvDefault>();
}

hipError_t chunked_set_attributes() {
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chain(set_attr_lpr<CE_PARTIAL, VK_F32X>());
  chain(set_attr_lpr<CE_PARTIAL, VK_BF16X>());
  chain(set_attr_lpr<CE_ROW, VK_F32X>());
  chain(set_attr_lpr<CE_ROW, VK_BF16X>());
  chain(set_attr_lpr<CE_COL, VK_F32X>());
  chain(set_attr_lpr<CE_COL, VK_BF16X>());
  chain(set_attr_lpr<CE_PARTIAL, VK_F64>());
  chain(set_attr_lpr<CE_PARTIAL, VK_F32>());
  chain(set_attr_lpr<CE_PARTIAL, VK_BF16>());
  chain(set_attr_lpr<CE_ROW, VK_F64>());
  chain(set_attr_lpr<CE_ROW, VK_F32>());
  chain(set_attr_lpr<CE_ROW, VK_BF16>());
  chain(set_attr_lpr<CE_COL, VK_F64>());
  chain(set_attr_lpr<CE_COL, VK_F32>());
  chain(set_attr_lpr<CE_COL, VK_BF16>());
  return e;
}

hipError_t launch_chunk_epilogue_col(const ChunkArgs& c, const ColArgs& ca, int grid, hipStream_t st,
                                     const KEvents* ev) {
  return launch_ev(ev, k_chunk_epilogue_col, dim3(grid), dim3(kBlock), 0, st, c, ca);
}

hipError_t launch_chunk_epilogue_row(const ChunkArgs& c, const RowArgs& ra, int grid, hipStream_t st,
                                     const KEvents* ev) {
  return launch_ev(ev, k_chunk_epilogue_row, dim3(grid), dim3(kBlock), 0, st, c, ra);
}

hipError_t launch_ts_reduce(int vk, const TsArgs& a, int grid, hipStream_t st, const KEvents* ev) {
  const dim3 g(grid), b(kBlock);
  if (vk == VK_F32) return launch_ev(ev, k_ts_reduce<VK_F32>, g, b, 0, st, a);
  if (vk == VK_BF16) return launch_ev(ev, k_ts_reduce<VK_BF16>, g, b, 0, st, a);
  if (vk == VK_F32X) return launch_ev(ev, k_ts_reduce<VK_F32X>, g, b, 0, st, a);
  if (vk == VK_BF16X) return launch_ev(ev, k_ts_reduce<VK_BF16X>, g, b, 0, st, a);
  return launch_ev(ev, k_ts_reduce<VK_F64>, g, b, 0, st, a);
}

hipError_t launch_ts_finish(int mode, const TsFinishArgs& a, hipStream_t st) {
  const int KW = a.k + a.me;
  if (KW == 0) return hipSuccess;
  if (mode == TS_MATVEC) k_ts_finish<TS_MATVEC><<<KW, kBlock, 0, st>>>(a);
  else if (mode == TS_RESID) k_ts_finish<TS_RESID><<<KW, kBlock, 0, st>>>(a);
  else k_ts_finish<TS_GONLY><<<KW, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_rhs_lam(const VecArgs& a, hipStream_t st) {
  if (a.me + a.m == 0) return hipSuccess;
  k_rhs_lam<<<grid_for(a.me + a.m, kBlock), kBlock, 0, st>>>(a);
  return hipGetLastError();
}
hipError_t launch_recover_x(const VecArgs& a, int grid, hipStream_t st) {
  k_recover_x<<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}
hipError_t launch_finish_ratio(const VecArgs& a, int g_r, int g_x, hipStream_t st) {
  k_finish_ratio<<<1, kBlock, 0, st>>>(a, g_r, g_x);
  return hipGetLastError();
}
hipError_t launch_finish_norms(const VecArgs& a, int g_r, int g_x, hipStream_t st) {
  k_finish_norms<<<1, kBlock, 0, st>>>(a, g_r, g_x);
  return hipGetLastError();
}
hipError_t launch_update(const VecArgs& a, const double* dx, const double* dlam, const double* ds,
                         const double* alpha_dev, double ax, double al, int grid, hipStream_t st) {
  k_update<<<grid, kBlock, 0, st>>>(a, dx, dlam, ds, alpha_dev, ax, al);
  return hipGetLastError();
}
hipError_t launch_init_x(const VecArgs& a, int grid, hipStream_t st) {
  k_init_x<<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}
hipError_t launch_check_state(const VecArgs& a, int grid, hipStream_t st) {
  k_check_state<<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}
hipError_t launch_finish_sum(const double* part, int count, double* out, hipStream_t st) {
  k_finish_sum<<<1, kBlock, 0, st>>>(part, count, out);
  return hipGetLastError();
}
hipError_t launch_cg_init(const CgArgs& a, hipStream_t st) {
  k_cg_init<<<a.g_vec, kBlock, 0, st>>>(a);
  k_cg_init_finish<<<1, kBlock, 0, st>>>(a);
  return hipGetLastError();
}
hipError_t launch_cg_update(const CgArgs& a, hipStream_t st, const KEvents* ev) {
  if (a.qpart) return launch_ev(ev, k_cg_update_split, dim3(a.g_vec), dim3(kBlock), 0, st, a);
  return launch_ev(ev, k_cg_update, dim3(a.g_vec), dim3(kBlock), 0, st, a);
}
hipError_t launch_compl(const VecArgs& a, const double* dlam, const double* ds, double* part0,
                        double* part1, double* part2, int grid, hipStream_t st) {
  k_compl<<<grid, kBlock, 0, st>>>(a, dlam, ds, part0, part1, part2);
  return hipGetLastError();
}
hipError_t launch_second_order(const VecArgs& a, double* res, const double* dlam, const double* ds,
                               int grid, hipStream_t st) {
  k_second_order<<<grid, kBlock, 0, st>>>(a, res, dlam, ds);
  return hipGetLastError();
}
hipError_t launch_cg_pupdate(const CgArgs& a, hipStream_t st, const KEvents* ev) {
  return launch_ev(ev, k_cg_pupdate, dim3(a.g_vec), dim3(kBlock), 0, st, a);
}
hipError_t launch_cg_restart(const CgArgs& a, const double* kx, int resume, hipStream_t st) {
  k_cg_restart<<<a.g_vec, kBlock, 0, st>>>(a, kx, resume);
  if (resume) k_cg_rearm<<<1, 64, 0, st>>>(a.fl);
  return hipGetLastError();
}
hipError_t launch_grad_out(int n, int m, int me, const double* u, const double* lA,
                           const double* uA, double* gc, double* glA, double* guA, double* gb,
                           hipStream_t st) {
  k_grad_out<<<grid_for(n > m ? n : m, kBlock), kBlock, 0, st>>>(n, m, me, u, lA, uA, gc, glA, guA, gb);
  return hipGetLastError();
}
hipError_t launch_copy(const double* src, double* dst, int64_t n, double scale, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_copy<<<grid_for(n, kBlock), kBlock, 0, st>>>(src, dst, n, scale);
  return hipGetLastError();
}
hipError_t launch_sqdiff(const double* a, const double* b, int64_t n, double* part, int grid,
                         hipStream_t st) {
  k_sqdiff<<<grid, kBlock, 0, st>>>(a, b, n, part);
  return hipGetLastError();
}
hipError_t launch_ratio_given(const VecArgs& a, const double* dlam, const double* ds, int grid,
                              hipStream_t st) {
  k_ratio_given<<<grid, kBlock, 0, st>>>(a, dlam, ds);
  return hipGetLastError();
}
hipError_t launch_fill(double* dst, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<grid_for(n, kBlock), kBlock, 0, st>>>(dst, n, v);
  return hipGetLastError();
}


// ------------------------------------------ fused pass launcher
constexpr int kFusedPP = 4;   // entry pairs per lane per batch: 64 entries per row

static uint32_t fused_lds(const FusedArgs& f) {
  return static_cast<uint32_t>(sizeof(double)) * (2u * f.half + kFusedOwn);
}

hipError_t launch_fused(int vk, const FusedArgs& f, const RowArgs& ra, hipStream_t st, const KEvents* ev) {
  const dim3 g(2 * f.nrange), b(kChunkBlock);
  const uint32_t lds = fused_lds(f);
  switch (vk) {
    case VK_F32: return launch_ev(ev, k_fused<VK_F32, kFusedPP>, g, b, lds, st, f, ra);
    case VK_BF16: return launch_ev(ev, k_fused<VK_BF16, kFusedPP>, g, b, lds, st, f, ra);
    case VK_F32X: return launch_ev(ev, k_fused<VK_F32X, kFusedPP>, g, b, lds, st, f, ra);
    case VK_BF16X: return launch_ev(ev, k_fused<VK_BF16X, kFusedPP>, g, b, lds, st, f, ra);
    default: return launch_ev(ev, k_fused<VK_F64, kFusedPP>, g, b, lds, st, f, ra);
  }
}

hipError_t fused_set_attributes() {
  const int lds = sizeof(double) * (2 * kFusedHalfMax + kFusedOwn);
  hipError_t e = hipSuccess;
  auto one = [&](const void* fn) {
    if (e == hipSuccess) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  };
  one(reinterpret_cast<const void*>(&k_fused<VK_F64, kFusedPP>));
  one(reinterpret_cast<const void*>(&k_fused<VK_F32, kFusedPP>));
  one(reinterpret_cast<const void*>(&k_fused<VK_BF16, kFusedPP>));
  one(reinterpret_cast<const void*>(&k_fused<VK_F32X, kFusedPP>));
  one(reinterpret_cast<const void*>(&k_fused<VK_BF16X, kFusedPP>));
  return e;
}

}  // namespace qpk
