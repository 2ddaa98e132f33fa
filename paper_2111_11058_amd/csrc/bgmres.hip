// Block GMRES: the right-hand sides of one operator (the incidences of a
// scatterer, Sec. III-C outer equation with many excitations) share one
// Krylov space K_J(A, R_0) built from the block of all their residuals, and
// each right-hand side's iterate minimises its own residual over the whole
// space.  Every iteration applies the operator to the p vectors of the last
// block (the same matrix-core product as p single-vector iterations) and
// adds p basis vectors; correlated right-hand sides (plane waves a degree or
// two apart) then converge in far fewer products than one at a time.
//
// Block Arnoldi with block classical Gram-Schmidt applied twice: pass 1
// projects the new block against the basis, an intra-block orthonormalisation
// follows, and pass 2 repeats both on the result, so that directions scaled
// up by the first normalisation lose what the first projection left of the
// basis.  The intra-block step is Cholesky QR on a Gram matrix accumulated in
// double-double arithmetic (Dekker's exact products and Knuth's two-sum),
// factored with diagonal pivoting in double-double: a block whose vectors
// are numerically dependent (the incidences' residuals are, to about 1e-10)
// keeps its independent directions down to a relative size of 1e-13 and
// gets random vectors in place of the rest; those have no coefficient in
// the Arnoldi relation, so the relation A V_J = V_{J+1} H still holds to
// rounding.
//
// The block Hessenberg matrix is reduced to triangular form as it grows: each
// new block column takes the unitary 2p x 2p factors of the earlier block
// rows in turn, and a Householder QR of its last 2p rows gives the next
// factor.  The same factors applied to E_1 S_0 (R_0 = V_0 S_0) leave every
// right-hand side's residual norm in the last p rows, which stops the cycle
// once all of them are below tol.  At the end of a cycle a back substitution
// gives Y and x += V Y; the next cycle, if any, starts from the true
// residual b - A x.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "gemm.h"
#include "solve.h"

namespace cbfm {
namespace {

constexpr int PMAX = 32;  // right-hand sides per block (a power of two: indices below use e >> 5)
static_assert(PMAX == 32, "index arithmetic assumes 32");
constexpr int GCH = 32;   // vector entries per block of the Gram partial sums
constexpr int OMS = 2 * PMAX;  // row stride of a stored 2p x 2p factor (zero past 2p)
constexpr int RBUF = 6144;     // rows of a block column staged in LDS (mb p <= RBUF)

__device__ inline double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 c_cjmul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// ---- double-double arithmetic: hi + lo with |lo| <= ulp(hi) / 2
struct dd {
  double hi, lo;
};
__device__ inline dd dd_two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd dd_fast_sum(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__device__ inline dd dd_prod(double a, double b) {  // exact product (one FMA)
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__device__ inline dd dd_add(dd a, dd b) {
  dd s = dd_two_sum(a.hi, b.hi);
  const dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast_sum(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast_sum(s.hi, s.lo);
}
__device__ inline dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
__device__ inline dd dd_mul(dd a, dd b) {
  dd p = dd_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_fast_sum(p.hi, p.lo);
}
__device__ inline dd dd_mul_d(dd a, double b) {
  dd p = dd_prod(a.hi, b);
  p.lo += a.lo * b;
  return dd_fast_sum(p.hi, p.lo);
}
__device__ inline dd dd_div(dd a, dd b) {  // three quotient digits
  const double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
  const double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
  const double q3 = r.hi / b.hi;
  return dd_add(dd_fast_sum(q1, q2), dd{q3, 0.0});
}
__device__ inline dd dd_sqrt(dd a) {  // one Newton step from the double root
  if (!(a.hi > 0)) return dd{0.0, 0.0};
  const double x = sqrt(a.hi);
  const dd r = dd_add(a, dd_neg(dd_prod(x, x)));
  return dd_fast_sum(x, r.hi / (2.0 * x));
}
struct cdd {
  dd re, im;
};

// Counter-based uniform numbers in (-1, 1): the splitmix64 output function
// (Steele, Lea and Flood, 2014) of a 64-bit counter.
__device__ inline double unit_random(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Cycle control on the device: [0] 0 running, 1 converged, 2 broken down;
// [1] block columns completed in this cycle.
enum { CTL_STATE = 0, CTL_DONE = 1 };

// ---- Gram partial sums: G[a][b] = sum_i conj(W[a][i]) W[b][i] for a <= b
// < p over the GCH entries of this block, real and imaginary parts in
// double-double (DD) or in double (low parts zero: the second pass, whose
// rows the first has made orthonormal to within about 1e-3 at worst); entry
// (a, b) at a * PMAX + b of the
// block's PMAX^2 slots.
template <bool DD>
__global__ void __launch_bounds__(256) gram_partial_kernel(const double2* __restrict__ W, int64_t n, int p,
                                                           double* __restrict__ part, const int32_t* __restrict__ ctl) {
  if (ctl[CTL_STATE] != 0) return;  // uniform over the launch
  __shared__ double2 ws[PMAX][GCH + 1];
  const int64_t i0 = (int64_t)blockIdx.x * GCH;
  for (int e = threadIdx.x; e < p * GCH; e += 256) {
    const int a = e / GCH, k = e % GCH;
    ws[a][k] = i0 + k < n ? W[a * n + i0 + k] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < p * p; e += 256) {
    const int a = e / p, b = e % p;
    if (a > b) continue;
    dd sr{0.0, 0.0}, si{0.0, 0.0};
    if (DD) {
      for (int k = 0; k < GCH; ++k) {
        const double2 x = ws[a][k], y = ws[b][k];
        sr = dd_add(sr, dd_add(dd_prod(x.x, y.x), dd_prod(x.y, y.y)));
        si = dd_add(si, dd_add(dd_prod(x.x, y.y), dd_prod(-x.y, y.x)));
      }
    } else {
#pragma unroll 8
      for (int k = 0; k < GCH; ++k) {
        const double2 x = ws[a][k], y = ws[b][k];
        sr.hi = fma(x.x, y.x, fma(x.y, y.y, sr.hi));
        si.hi = fma(x.x, y.y, fma(-x.y, y.x, si.hi));
      }
    }
    double* o = part + ((int64_t)blockIdx.x * PMAX * PMAX + a * PMAX + b) * 4;
    o[0] = sr.hi;
    o[1] = sr.lo;
    o[2] = si.hi;
    o[3] = si.lo;
  }
}

// ---- The partial sums of every Gram entry added over the nchunk blocks in
// double-double: one wavefront per entry (a, b), a <= b, lanes taking every
// 64th block, then a butterfly over the lanes.
__global__ void __launch_bounds__(256) gram_reduce_kernel(const double* __restrict__ part, int nchunk, int p,
                                                          double* __restrict__ G, const int32_t* __restrict__ ctl) {
  if (ctl[CTL_STATE] != 0) return;  // uniform over the launch
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= p * p) return;  // uniform over the wavefront
  const int a = e / p, b = e % p;
  if (a > b) return;
  const int slot = a * PMAX + b;
  dd sr{0.0, 0.0}, si{0.0, 0.0};
  for (int c = lane; c < nchunk; c += 64) {
    const double* o = part + ((int64_t)c * PMAX * PMAX + slot) * 4;
    sr = dd_add(sr, dd{o[0], o[1]});
    si = dd_add(si, dd{o[2], o[3]});
  }
  for (int off = 32; off >= 1; off >>= 1) {
    sr = dd_add(sr, dd{__shfl_xor(sr.hi, off), __shfl_xor(sr.lo, off)});
    si = dd_add(si, dd{__shfl_xor(si.hi, off), __shfl_xor(si.lo, off)});
  }
  if (lane == 0) {
    double* g = G + slot * 4;
    g[0] = sr.hi;
    g[1] = sr.lo;
    g[2] = si.hi;
    g[3] = si.lo;
  }
}

// ---- Pivoted Cholesky of the Gram matrix in double-double (one block).
// G = R^H R with the pivot of step k the remaining column of largest Schur
// diagonal, while that diagonal exceeds tau times the largest diagonal of G
// (rank r = the steps taken).  Outputs (double, p x p, row-major):
//   M[l][a]: W[a] = sum_{l<r} M[l][a] q_l (rows l >= r zero),
//   T[a][l]: q_l = sum_a T[a][l] W[a] for l < r (T = the inverse of R's
//            pivoted r x r triangle, scattered to the pivot rows),
//   rank[0] = r.  With must_full, r < p marks the cycle broken down.
__global__ void __launch_bounds__(256) chol_pivot_kernel(const double* __restrict__ Gdd, int p, double tau,
                                                         double2* __restrict__ M, double2* __restrict__ T,
                                                         int32_t* __restrict__ rank, int32_t* __restrict__ ctl,
                                                         int must_full) {
  if (ctl[CTL_STATE] != 0) return;  // uniform over the launch
  __shared__ cdd S[PMAX][PMAX];      // Schur complement (entries a <= b)
  __shared__ double2 R[PMAX][PMAX];  // rows of R (double)
  __shared__ cdd Rk[PMAX];           // the current row of R
  __shared__ double2 U[PMAX][PMAX];  // inverse of the pivoted triangle
  __shared__ int piv[PMAX], used[PMAX], pos[PMAX];
  __shared__ int q_s, r_s, redo_s;
  __shared__ double dmax0;
  const int tid = threadIdx.x;
  for (int e = tid; e < PMAX * PMAX; e += 256) {
    const int a = e >> 5, b = e & (PMAX - 1);
    if (a >= p || b >= p) continue;
    if (a <= b) {
      const double* g = Gdd + (a * PMAX + b) * 4;
      S[a][b] = cdd{dd{g[0], g[1]}, dd{g[2], g[3]}};
    }
  }
  for (int e = tid; e < PMAX * PMAX; e += 256) {
    R[e / PMAX][e % PMAX] = make_double2(0.0, 0.0);
    U[e / PMAX][e % PMAX] = make_double2(0.0, 0.0);
  }
  if (tid < PMAX) {
    used[tid] = 0;
    pos[tid] = -1;
  }
  __syncthreads();
  if (tid < 64) {  // largest diagonal (wavefront 0)
    double m = tid < p ? S[tid][tid].re.hi : 0.0;
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (tid == 0) {
      dmax0 = m;
      r_s = p;
      redo_s = 0;
    }
  }
  __syncthreads();
  // First in double, without pivoting, on the Gram matrix with unit
  // diagonal (columns of W scaled to unit norm, which leaves Q unchanged):
  // accepted when no column of W is below 1e-10 of the largest in norm and
  // every pivot of the scaled matrix stays above 1e-10 (its condition below
  // 1e5, where Cholesky QR in double loses at most about 1e-6 of
  // orthogonality, which the second pass restores); otherwise the
  // factorisation is redone in double-double with pivoting.  One barrier
  // per step: each thread takes the pivot row from the matrix itself.
  {
    double2(*Sd)[PMAX] = U;  // U is free until the inverse
    __shared__ double dsc[PMAX];
    if (tid < p) {
      const double d = S[tid][tid].re.hi + S[tid][tid].re.lo;
      dsc[tid] = d > 0 ? sqrt(d) : 0.0;
      if (!(d >= 1e-20 * dmax0)) redo_s = 1;
    }
    __syncthreads();
    for (int e = tid; e < PMAX * PMAX; e += 256) {
      const int a = e >> 5, b = e & (PMAX - 1);
      if (a >= p || b >= p) continue;
      if (a <= b && !redo_s) {
        const double sc = 1.0 / (dsc[a] * dsc[b]);
        Sd[a][b] = make_double2((S[a][b].re.hi + S[a][b].re.lo) * sc, (S[a][b].im.hi + S[a][b].im.lo) * sc);
      }
    }
    __syncthreads();
    for (int k = 0; k < p && !redo_s; ++k) {  // redo_s: uniform after each barrier
      const double pk = Sd[k][k].x;
      if (!(pk > 1e-10)) {
        if (tid == 0) redo_s = 1;
        __syncthreads();
        break;
      }
      const double sq = sqrt(pk), inv = 1.0 / pk;
      if (tid < p) {  // row k of the scaled factor, unscaled by the column norm
        const int m = tid;
        const double2 v = m < k ? make_double2(0.0, 0.0) : (m == k ? make_double2(sq, 0.0) : Sd[k][m]);
        const double f = (m == k ? 1.0 : 1.0 / sq) * dsc[m];
        R[k][m] = make_double2(v.x * f, v.y * f);
      }
      for (int e = tid; e < PMAX * PMAX; e += 256) {  // Schur update of the trailing pairs
        const int a = e >> 5, b = e & (PMAX - 1);
        if (a <= k || a > b || b >= p) continue;
        const double2 t = c_cjmul(Sd[k][a], Sd[k][b]);
        Sd[a][b] = make_double2(Sd[a][b].x - t.x * inv, Sd[a][b].y - t.y * inv);
      }
      __syncthreads();
    }
    if (!redo_s && tid < p) {
      piv[tid] = tid;
      pos[tid] = tid;
      used[tid] = 1;
    }
    if (redo_s) {  // uniform: start again in double-double
      for (int e = tid; e < PMAX * PMAX; e += 256) {
        R[e / PMAX][e % PMAX] = make_double2(0.0, 0.0);
        U[e / PMAX][e % PMAX] = make_double2(0.0, 0.0);
      }
      if (tid < PMAX) {
        used[tid] = 0;
        pos[tid] = -1;
      }
    }
    __syncthreads();
  }
  for (int k = 0; k < p && redo_s; ++k) {
    if (tid < 64) {  // pivot: the largest remaining diagonal, lowest index on ties
      double v = tid < p && !used[tid] ? S[tid][tid].re.hi : -1.0;
      int qi = tid;
      for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off);
        const int oq = __shfl_xor(qi, off);
        if (ov > v || (ov == v && oq < qi)) {
          v = ov;
          qi = oq;
        }
      }
      if (tid == 0) {
        if (!(v > tau * dmax0) || !(v > 0.0)) {
          r_s = k;
          q_s = -1;
        } else {
          used[qi] = 1;
          piv[k] = qi;
          pos[qi] = k;
          q_s = qi;
        }
      }
    }
    __syncthreads();
    const int q = q_s;
    if (q < 0) break;  // uniform
    if (tid < p) {     // row k of R over the remaining columns
      const int m = tid;
      cdd v{dd{0.0, 0.0}, dd{0.0, 0.0}};
      if (m == q) {
        v.re = dd_sqrt(S[q][q].re);
      } else if (!used[m]) {
        const dd rkk = dd_sqrt(S[q][q].re);
        // S[q][m] from the stored triangle (conjugate when m < q)
        const cdd sq = q <= m ? S[q][m] : cdd{S[m][q].re, dd_neg(S[m][q].im)};
        v.re = dd_div(sq.re, rkk);
        v.im = dd_div(sq.im, rkk);
      }
      Rk[m] = v;
      R[k][m] = make_double2(v.re.hi + v.re.lo, v.im.hi + v.im.lo);
    }
    __syncthreads();
    for (int e = tid; e < PMAX * PMAX; e += 256) {  // Schur update of the remaining pairs
      const int a = e >> 5, b = e & (PMAX - 1);
      if (a > b || b >= p || used[a] || used[b]) continue;
      const cdd x = Rk[a], y = Rk[b];
      // S[a][b] -= conj(x) y
      const dd pr = dd_add(dd_mul(x.re, y.re), dd_mul(x.im, y.im));
      const dd pi = dd_add(dd_mul(x.re, y.im), dd_neg(dd_mul(x.im, y.re)));
      S[a][b].re = dd_add(S[a][b].re, dd_neg(pr));
      S[a][b].im = dd_add(S[a][b].im, dd_neg(pi));
    }
    __syncthreads();
  }
  const int r = r_s;
  // U = inverse of Rp (Rp[j][k] = R[j][piv[k]], r x r upper triangular):
  // Rp gathered first (into Rk's rows of S, now free), then thread k takes
  // column k, rows from k down to 0
  double2(*Rp)[PMAX] = reinterpret_cast<double2(*)[PMAX]>(&S[0][0]);
  for (int e = tid; e < PMAX * PMAX; e += 256) {
    const int j = e >> 5, l = e & (PMAX - 1);
    if (j < r && l < r) Rp[j][l] = R[j][piv[l]];
  }
  for (int e = tid; e < PMAX * PMAX; e += 256) U[e / PMAX][e % PMAX] = make_double2(0.0, 0.0);
  __syncthreads();
  if (tid < r) {
    const int k = tid;
    for (int j = k; j >= 0; --j) {
      double2 s = make_double2(j == k ? 1.0 : 0.0, 0.0);
#pragma unroll 8
      for (int l = j + 1; l <= k; ++l) s = c_sub(s, c_mul(Rp[j][l], U[l][k]));
      const double d = Rp[j][j].x;  // real and positive
      U[j][k] = make_double2(s.x / d, s.y / d);
    }
  }
  __syncthreads();
  for (int e = tid; e < PMAX * PMAX; e += 256) {
    const int l = e >> 5, a = e & (PMAX - 1);
    if (l < p && a < p) M[l * p + a] = l < r ? R[l][a] : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < PMAX * PMAX; e += 256) {
    const int a = e >> 5, l = e & (PMAX - 1);
    if (a >= p || l >= p) continue;
    const int j = pos[a];  // pivot position of row a, or -1
    T[a * p + l] = l < r && j >= 0 && j <= l ? U[j][l] : make_double2(0.0, 0.0);
  }
  if (tid == 0) {
    rank[0] = r;
    if (must_full && r < p) ctl[CTL_STATE] = 2;
  }
}

// ---- Out = the orthonormalised rows of W: row l < r is sum_a T[a][l] W[a],
// rows l >= r random (entries of modulus about 1 / sqrt(n)).  A thread takes
// one vector entry and 8 output rows (blockIdx.y picks them).
__global__ void __launch_bounds__(256) ortho_apply_kernel(const double2* __restrict__ W, double2* __restrict__ Out,
                                                          int64_t n, int p, const double2* __restrict__ T,
                                                          const int32_t* __restrict__ rank, uint64_t seed,
                                                          const int32_t* __restrict__ ctl) {
  if (ctl[CTL_STATE] != 0) return;  // uniform over the launch
  __shared__ double2 Ts[PMAX][8];
  const int l0 = blockIdx.y * 8;
  for (int e = threadIdx.x; e < p * 8; e += 256) {
    const int a = e / 8, u = e % 8;
    Ts[a][u] = l0 + u < p ? T[a * p + l0 + u] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int r = rank[0];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double2 o[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) o[u] = make_double2(0.0, 0.0);
  for (int a = 0; a < p; ++a) {
    const double2 w = W[a * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) o[u] = c_add(o[u], c_mul(Ts[a][u], w));
  }
  const double sc = sqrt(1.5 / (double)n);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int l = l0 + u;
    if (l >= p) break;
    if (l >= r) {
      const uint64_t z = (seed * 64 + (uint64_t)l) * 0x100000000ull + (uint64_t)i;
      o[u] = make_double2(sc * unit_random(2 * z), sc * unit_random(2 * z + 1));
    }
    Out[l * n + i] = o[u];
  }
}

// ---- S0 = M2 M1 into rows 0..p-1 of G (the initial block's coefficients,
// R_0 = V_0 S0); the rest of G zero.
__global__ void s0_kernel(const double2* __restrict__ M1, const double2* __restrict__ M2, int p, double2* __restrict__ G,
                          int64_t grows) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= grows * p) return;
  const int64_t k = e / p;
  const int c = (int)(e % p);
  double2 v = make_double2(0.0, 0.0);
  if (k < p)
    for (int l = 0; l < p; ++l) v = c_add(v, c_mul(M2[k * p + l], M1[l * p + c]));
  G[e] = v;
}

// ---- Block column J of the Hessenberg matrix for right-hand-side column c
// (one block per column): H[k][c] = C1[k][c] + sum_l C2[k][l] M1[l][c] for
// k < (J+1)p and (M2 M1)[m][c] in rows (J+1)p + m; then the unitary factors
// of block rows 0..J-1 in turn (Om[i] = Omega_i^H acts on rows ip..ip+2p-1).
// Rows below Jp are final: they go to column Jp + c of Rb (column-major,
// ldr; staged in LDS, Jp <= RBUF); rows Jp..Jp+2p-1 go to the slab X
// (2p x p) for the QR of this block.
__global__ void __launch_bounds__(256) bls_column_kernel(const double2* __restrict__ C1, const double2* __restrict__ C2,
                                                         const double2* __restrict__ M1,
                                                         const double2* __restrict__ M2,
                                                         const double2* __restrict__ Om, int64_t J, int p,
                                                         double2* __restrict__ h, int64_t hstride,
                                                         double2* __restrict__ Rb, int64_t ldr,
                                                         double2* __restrict__ X, const int32_t* __restrict__ ctl) {
  if (ctl[CTL_STATE] != 0) return;  // uniform over the launch
  const int c = blockIdx.x, tid = threadIdx.x;
  __shared__ double2 m1[PMAX];
  __shared__ double2 slab[2 * PMAX + 1];
  __shared__ double2 fin[RBUF];  // the column's final rows 0..Jp-1, stored at the end
  if (tid < p) m1[tid] = M1[tid * p + c];
  if (tid < 2 * PMAX) slab[tid] = make_double2(0.0, 0.0);
  __syncthreads();
  double2* hc = h + c * hstride;  // this column's work vector in global memory
  const int64_t top = (J + 1) * p;
  for (int64_t k = tid; k < top + p; k += 256) {
    const double2* row = k < top ? C2 + k * p : M2 + (k - top) * p;
    double2 cr[PMAX];
#pragma unroll
    for (int l = 0; l < PMAX; ++l) cr[l] = l < p ? row[l] : make_double2(0.0, 0.0);
    double2 v = k < top ? C1[k * p + c] : make_double2(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < PMAX; ++l)
      if (l < p) v = c_add(v, c_mul(cr[l], m1[l]));
    hc[k] = v;
  }
  __syncthreads();
  const int p2 = 2 * p;
  // factors of the earlier block rows: 4 threads per row of the slab, each
  // summing every 4th of the 2p columns; the next factor's rows are loaded
  // while the current one is applied
  const int row = tid >> 2, qtr = tid & 3;
  // (factor rows are OMS long and zero past 2p, so the loads and products
  // below need no conditions)
  auto load = [&](int64_t i, double2(&o)[16]) {
    const double2* op = Om + (size_t)i * OMS * OMS + (size_t)row * OMS;
#pragma unroll
    for (int u = 0; u < 16; ++u) o[u] = op[qtr + 4 * u];
  };
  // one step of the factors: slab <- Omega_i^H slab with the factor's rows
  // in o and the next half of the slab in hn
  auto step = [&](int64_t i, const double2(&o)[16], double2 hn) {
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 16; ++u) s = c_add(s, c_mul(o[u], slab[qtr + 4 * u]));
    s.x += __shfl_xor(s.x, 1);
    s.y += __shfl_xor(s.y, 1);
    s.x += __shfl_xor(s.x, 2);
    s.y += __shfl_xor(s.y, 2);
    __syncthreads();  // every read of the slab done
    if (row < p2 && qtr == 0) {
      if (row < p)
        fin[i * p + row] = s;  // final row i p + row
      else
        slab[row - p] = s;  // carried into the next block row
    }
    if (tid < p) slab[p + tid] = hn;
    __syncthreads();
  };
  // two register sets in turn, so that the loads of a factor are two steps
  // ahead of its use
  const int tc = tid < p ? tid : p - 1;  // (threads past p load a valid entry, unused)
  auto hload = [&](int64_t i) { return hc[(i + 2) * p + tc]; };
  double2 oA[16], oB[16], hA = make_double2(0.0, 0.0), hB = make_double2(0.0, 0.0);
  if (tid < p2) slab[tid] = hc[tid];
  if (J > 0) {
    load(0, oA);
    hA = hload(0);
  }
  if (J > 1) {
    load(1, oB);
    hB = hload(1);
  }
  __syncthreads();
  for (int64_t i = 0; i < J; i += 2) {
    step(i, oA, hA);
    if (i + 2 < J) {
      load(i + 2, oA);
      hA = hload(i + 2);
    }
    if (i + 1 < J) {
      step(i + 1, oB, hB);
      if (i + 3 < J) {
        load(i + 3, oB);
        hB = hload(i + 3);
      }
    }
  }
  for (int64_t k = tid; k < J * p; k += 256) Rb[(J * p + c) * ldr + k] = fin[k];
  if (tid < p2) X[tid * p + c] = slab[tid];
}

// ---- Householder QR of the slab X (2p x p) of block column J (one block):
// Omega_J^H X = [R_JJ; 0].  R_JJ goes to Rb, Omega_J^H to Om[J] (rows of
// OMS entries, zero past 2p), and it is
// applied to rows Jp..Jp+2p-1 of G; the last p rows of G then hold every
// right-hand side's residual, whose norm relative to bnorm decides
// convergence (all <= tol).
__global__ void __launch_bounds__(256) bls_qr_kernel(const double2* __restrict__ X, int64_t J, int p,
                                                     double2* __restrict__ Rb, int64_t ldr, double2* __restrict__ Om,
                                                     double2* __restrict__ G, const double* __restrict__ bnorm,
                                                     double tol, double* __restrict__ res, int32_t* __restrict__ ctl) {
  if (ctl[CTL_STATE] != 0) return;  // uniform over the launch
  const int tid = threadIdx.x, p2 = 2 * p;
  __shared__ double2 A[2 * PMAX][PMAX + 1];        // the slab, reduced in place
  __shared__ double2 Q[2 * PMAX][2 * PMAX + 1];    // Omega^H, built up
  __shared__ double2 Gs[2 * PMAX][PMAX + 1];       // rows Jp.. of G
  __shared__ double2 v[2 * PMAX];
  __shared__ double beta_s;
  for (int e = tid; e < p2 * p; e += 256) {
    A[e / p][e % p] = X[e];
    Gs[e / p][e % p] = G[(J * p) * p + e];
  }
  for (int e = tid; e < p2 * p2; e += 256) Q[e / p2][e % p2] = make_double2(e / p2 == e % p2 ? 1.0 : 0.0, 0.0);
  __syncthreads();
  const int ncol = 4 * p;  // columns updated per reflector: A (p), Q (2p), Gs (p)
  for (int k = 0; k < p; ++k) {
    if (tid < 64) {  // reflector of column k (rows k..2p-1), wave 0
      double s2 = 0.0;
      for (int r = k + tid; r < p2; r += 64) s2 += A[r][k].x * A[r][k].x + A[r][k].y * A[r][k].y;
      for (int o = 32; o >= 1; o >>= 1) s2 += __shfl_xor(s2, o);
      const double nrm = sqrt(s2);
      const double2 x0 = A[k][k];
      const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      // alpha = -e^{i arg x0} |x|, v = x - alpha e_k
      const double2 ph = a0 > 0 ? make_double2(x0.x / a0, x0.y / a0) : make_double2(1.0, 0.0);
      const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
      for (int r = tid; r < p2; r += 64) v[r] = r < k ? make_double2(0.0, 0.0) : (r == k ? c_sub(x0, alpha) : A[r][k]);
      // |v|^2 = |x|^2 - |x0|^2 + |x0 - alpha|^2 = 2 |x| (|x| + |x0|)
      const double vn = 2.0 * nrm * (nrm + a0);
      if (tid == 0) beta_s = vn > 0 ? 2.0 / vn : 0.0;
    }
    __syncthreads();
    const double beta = beta_s;
    // apply I - beta v v^H to the columns: 2 threads per column
    {
      const int col = tid >> 1, half = tid & 1;
      double2* base = nullptr;
      int stride = 0, cidx = 0;
      if (col < p) {
        base = &A[0][0];
        stride = PMAX + 1;
        cidx = col;
      } else if (col < 3 * p) {
        base = &Q[0][0];
        stride = 2 * PMAX + 1;
        cidx = col - p;
      } else if (col < ncol) {
        base = &Gs[0][0];
        stride = PMAX + 1;
        cidx = col - 3 * p;
      }
      double2 s = make_double2(0.0, 0.0);
      if (base && beta != 0.0)
#pragma unroll 8
        for (int r = k + half; r < p2; r += 2) s = c_add(s, c_cjmul(v[r], base[r * stride + cidx]));
      s.x += __shfl_xor(s.x, 1);
      s.y += __shfl_xor(s.y, 1);
      // (each column is read and written by its own two threads only; the
      // reflector itself sits in v)
      if (base && beta != 0.0)
#pragma unroll 8
        for (int r = k + half; r < p2; r += 2) {
          const double2 t = c_mul(v[r], make_double2(beta * s.x, beta * s.y));
          base[r * stride + cidx] = c_sub(base[r * stride + cidx], t);
        }
    }
    __syncthreads();
  }
  for (int e = tid; e < p * p; e += 256) {
    const int r = e / p, c = e % p;
    Rb[(J * p + c) * ldr + J * p + r] = r <= c ? A[r][c] : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < OMS * OMS; e += 256) {
    const int r = e / OMS, k = e % OMS;
    Om[(size_t)J * OMS * OMS + e] = r < p2 && k < p2 ? Q[r][k] : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < p2 * p; e += 256) G[(J * p) * p + e] = Gs[e / p][e % p];
  __shared__ int conv;
  if (tid == 0) conv = 1;
  __syncthreads();
  if (tid < p) {
    double s2 = 0.0;
    for (int r = p; r < p2; ++r) s2 += Gs[r][tid].x * Gs[r][tid].x + Gs[r][tid].y * Gs[r][tid].y;
    const double rr = bnorm[tid] > 0 ? sqrt(s2) / bnorm[tid] : 0.0;
    res[tid] = rr;
    if (!(rr <= tol)) atomicAnd(&conv, 0);
  }
  __syncthreads();
  if (tid == 0) {
    ctl[CTL_DONE] = (int32_t)(J + 1);
    if (conv) ctl[CTL_STATE] = 1;
  }
}

// ---- One step of the block back substitution Y = R^{-1} G (R upper
// triangular, column-major with ldr, in p x p diagonal blocks; G and Y
// row-major, p columns): every block solves the diagonal block b for all p
// columns (thread c takes column c; a zero diagonal, a direction with no
// part in the least-squares solution, gives a zero entry), block (0, 0)
// stores Y_b, and each thread then removes R[k][block b] Y_b from its row
// k < b p of G, in the eight columns of its blockIdx.y.
__global__ void __launch_bounds__(256) backsolve_step_kernel(const double2* __restrict__ Rb, int64_t ldr,
                                                             double2* __restrict__ G, int p, int64_t b,
                                                             double2* __restrict__ Y) {
  __shared__ double2 Rbb[PMAX][PMAX + 1];
  __shared__ double2 yb[PMAX][PMAX + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = b * p;
  for (int e = tid; e < p * p; e += 256) {
    const int r = e % p, k = e / p;  // column k of the block, row r
    Rbb[r][k] = Rb[(r0 + k) * ldr + r0 + r];
  }
  for (int e = tid; e < p * p; e += 256) yb[e / p][e % p] = G[(r0 + e / p) * p + e % p];
  __syncthreads();
  if (tid < p) {
    const int c = tid;
    for (int r = p - 1; r >= 0; --r) {
      double2 g = yb[r][c];
#pragma unroll 8
      for (int k = r + 1; k < p; ++k) g = c_sub(g, c_mul(Rbb[r][k], yb[k][c]));
      const double2 d = Rbb[r][r];
      const double dn = d.x * d.x + d.y * d.y;
      yb[r][c] = dn > 0 ? make_double2((g.x * d.x + g.y * d.y) / dn, (g.y * d.x - g.x * d.y) / dn)
                        : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int e = tid; e < p * p; e += 256) Y[(r0 + e / p) * p + e % p] = yb[e / p][e % p];
  // row k, the eight columns c0..c0+7 of blockIdx.y
  const int64_t k = (int64_t)blockIdx.x * 256 + tid;
  const int c0 = blockIdx.y * 8;
  if (k >= r0 || c0 >= p) return;
  double2 acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < p; j0 += 8) {  // eight loads of the row in flight at a time
    double2 rv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) rv[u] = j0 + u < p ? Rb[(r0 + j0 + u) * ldr + k] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u < p ? j0 + u : j0;  // rv[u] is zero past p
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = c_add(acc[c], c_mul(rv[u], yb[j][c0 + c]));
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (c0 + c < p) G[k * p + c0 + c] = c_sub(G[k * p + c0 + c], acc[c]);
}

__global__ void __launch_bounds__(256) vec_norms_kernel(const double2* __restrict__ u, int64_t n,
                                                        double* __restrict__ out) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double2 v = u[c * n + i];
    s += v.x * v.x + v.y * v.y;
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sqrt(red[0]);
}

__global__ void sub_from_b_kernel(const double2* __restrict__ b, double2* __restrict__ r, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < total) r[e] = c_sub(b[e], r[e]);
}

__global__ void ctl_reset_kernel(int32_t* ctl) {
  ctl[CTL_STATE] = 0;
  ctl[CTL_DONE] = 0;
}

// One group of p <= PMAX right-hand sides (rows of b and x, n entries each).
// The block of an iteration is formed in two work blocks before it enters
// the basis: t1 = A V_J, projected; t2 = its orthonormalised rows,
// projected again; slot J + 1 = the orthonormalised rows of t2.
class BlockGmres {
 public:
  BlockGmres(const double2* A, int64_t lda, const float2* A32, int64_t lda32, int64_t n, int p, int64_t mb,
             hipStream_t s)
      : A_(A), lda_(lda), A32_(A32), lda32_(lda32), n_(n), p_(p), mb_(mb), s_(s), nch_((int)((n + GCH - 1) / GCH)),
        V_((size_t)(mb + 1) * p * n * sizeof(double2), s), C1_(2 * (size_t)(mb + 1) * p * p * sizeof(double2), s),
        C2_(2 * (size_t)(mb + 1) * p * p * sizeof(double2), s), M1_(2 * p * p * sizeof(double2), s),
        M2_(2 * p * p * sizeof(double2), s), T_(p * p * sizeof(double2), s), rank_(sizeof(int32_t), s),
        part_((size_t)nch_ * PMAX * PMAX * 4 * sizeof(double), s), gdd_(PMAX * PMAX * 4 * sizeof(double), s),
        G_((size_t)(mb + 1) * p * p * sizeof(double2), s), Rb_((size_t)mb * p * mb * p * sizeof(double2), s),
        Om_((size_t)mb * OMS * OMS * sizeof(double2), s), h_((size_t)p * (mb + 2) * p * sizeof(double2), s),
        X_((size_t)2 * p * p * sizeof(double2), s), Y_((size_t)mb * p * p * sizeof(double2), s),
        bnorm_(p * sizeof(double), s), res_(p * sizeof(double), s), ctl_(2 * sizeof(int32_t), s),
        t1_((size_t)p * n * sizeof(double2), s), t2_((size_t)p * n * sizeof(double2), s) {
    std::vector<std::vector<GemmDesc>> mv(A_ ? mb : 0), upd(2 * mb);
    std::vector<std::vector<GemmDescX>> mvx(A_ ? 0 : mb);
    double2* V = V_.as<double2>();
    double2* t1 = t1_.as<double2>();
    double2* t2 = t2_.as<double2>();
    for (int64_t J = 0; J < mb; ++J) {
      if (A_) {
        GemmDesc d = gemm(A_, lda_, OP_N, V + J * p * n, n, OP_T, t1, n, n, p, n);
        d.transC = 1;
        mv[J].push_back(d);
      } else {  // a float operator: the product on the FP32 matrix cores, vectors in double
        GemmDescX d = gemmx(A32_, 0, lda32_, OP_N, V + J * p * n, 1, n, OP_T, t1, 1, n, n, p, n);
        d.transC = 1;
        mvx[J].push_back(d);
      }
      for (int ps = 0; ps < 2; ++ps) {
        double2* C = ps == 0 ? C1(J & 1) : C2(J & 1);
        double2* t = ps == 0 ? t1 : t2;
        dots_.push_back(gemm(V, n, OP_R, t, n, OP_T, C, p, (J + 1) * p, p, n));
        upd[2 * J + ps].push_back(gemm(C, p, OP_T, V, n, OP_N, t, n, p, n, (J + 1) * p, -1.0, 1));
      }
    }
    size_t ws = 1;
    for (const GemmDesc& d : dots_) ws = std::max(ws, panel_batch_ws_bytes(d, 1));
    dots_dev_.reset(new Scratch(std::max<size_t>(1, dots_.size()) * sizeof(GemmDesc), s));
    if (!dots_.empty()) {
      CBFM_HIP(hipMemcpyAsync(dots_dev_->p, dots_.data(), dots_.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
      CBFM_HIP(hipStreamSynchronize(s));
    }
    dots_ws_.reset(new Scratch(ws, s));
    if (A_)
      mv_.reset(new GemmPlan(mv, s));
    else
      mvx_.reset(new XGemmPlan(mvx, XG_FP32, s));
    upd_.reset(new GemmPlan(upd, s, false));
    CBFM_HIP(hipStreamCreateWithFlags(&ls_, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
      CBFM_HIP(hipEventCreateWithFlags(&ev_ready_[k], hipEventDisableTiming));
      CBFM_HIP(hipEventCreateWithFlags(&ev_read_[k], hipEventDisableTiming));
    }
  }
  ~BlockGmres() {
    if (ls_) {
      (void)hipStreamSynchronize(ls_);
      (void)hipStreamDestroy(ls_);
    }
    for (int k = 0; k < 2; ++k) {
      if (ev_ready_[k]) (void)hipEventDestroy(ev_ready_[k]);
      if (ev_read_[k]) (void)hipEventDestroy(ev_read_[k]);
    }
  }
  BlockGmres(const BlockGmres&) = delete;
  BlockGmres& operator=(const BlockGmres&) = delete;

  // Solve for the p right-hand sides b (rows) into x (rows, starting at 0).
  void solve(const double2* b, double2* x, double tol, int64_t max_iter, int64_t& total, std::vector<double>& res,
             bool& noconv) {
    const int p = p_;
    const int64_t n = n_;
    hipStream_t s = s_;
    double2* V = V_.as<double2>();
    double2* t1 = t1_.as<double2>();
    // t1 = A x (the operator's matrix-vector product shape, tuned)
    std::vector<std::vector<GemmDesc>> rg(A_ ? 1 : 0);
    std::vector<std::vector<GemmDescX>> rgx(A_ ? 0 : 1);
    if (A_) {
      rg[0].push_back(gemm(A_, lda_, OP_N, x, n, OP_T, t1, n, n, p, n));
      rg[0][0].transC = 1;
    } else {
      rgx[0].push_back(gemmx(A32_, 0, lda32_, OP_N, x, 1, n, OP_T, t1, 1, n, n, p, n));
      rgx[0][0].transC = 1;
    }
    const GemmPlan resid(rg, s);
    const XGemmPlan resid32(rgx, XG_FP32, s);
    auto residual = [&]() {  // t1 = b - A x
      if (A_)
        resid.launch(0, s);
      else
        resid32.launch(0, s);
      const int64_t tot = (int64_t)p * n;
      hipLaunchKernelGGL(sub_from_b_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, b, t1, tot);
      CBFM_HIP(hipGetLastError());
    };
    CBFM_HIP(hipMemsetAsync(x, 0, (size_t)p * n * sizeof(double2), s));
    hipLaunchKernelGGL(vec_norms_kernel, dim3((unsigned)p), dim3(256), 0, s, b, n, bnorm_.as<double>());
    PinnedFlags flags(1);
    int cycle = 0;
    for (;;) {
      if (cycle == 0)
        CBFM_HIP(hipMemcpyAsync(t1, b, (size_t)p * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
      else
        residual();
      hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(1), 0, s, ctl_.as<int32_t>());
      // R_0 = V_0 S0: two orthonormalisation passes into slot 0
      orthonormalise(t1, t2_.as<double2>(), M1(0), seed(cycle, 0, 0), false);
      orthonormalise(t2_.as<double2>(), V, M2(0), seed(cycle, 0, 1), true);
      const int64_t grows = (mb_ + 1) * p;
      hipLaunchKernelGGL(s0_kernel, dim3((unsigned)((grows * p + 255) / 256)), dim3(256), 0, s, M1(0), M2(0), p,
                         G_.as<double2>(), grows);
      CBFM_HIP(hipGetLastError());
      const int64_t mbc = std::min<int64_t>(mb_, max_iter - total);
      bool pending = false;
      for (int64_t J = 0; J < mbc; ++J) {
        iteration(J, cycle);
        ++total;
        if (pending && flags.wait()[0] != 0) break;
        flags.post(ctl_.as<int32_t>() + CTL_STATE, ls_);  // set by the least-squares stream
        pending = true;
      }
      CBFM_HIP(hipStreamSynchronize(ls_));
      int32_t ctl[2];
      CBFM_HIP(hipMemcpyAsync(ctl, ctl_.p, sizeof(ctl), hipMemcpyDeviceToHost, s));
      CBFM_HIP(hipStreamSynchronize(s));
      const int64_t nb = ctl[CTL_DONE], K = nb * p;
      if (K > 0) {
        for (int64_t bb = nb - 1; bb >= 0; --bb)
          hipLaunchKernelGGL(backsolve_step_kernel,
                             dim3((unsigned)std::max<int64_t>(1, (bb * p + 255) / 256), (unsigned)((p + 7) / 8)),
                             dim3(256), 0, s, Rb_.as<double2>(), mb_ * p, G_.as<double2>(), p, bb, Y_.as<double2>());
        CBFM_HIP(hipGetLastError());
        // x += Y^T V_0..V_{nb-1}
        std::vector<std::vector<GemmDesc>> xg(1);
        xg[0].push_back(gemm(Y_.as<double2>(), p, OP_T, V, n, OP_N, x, n, p, n, K, 1.0, 1));
        const GemmPlan xup(xg, s, false);
        xup.launch(0, s);
      }
      // true relative residuals
      residual();
      hipLaunchKernelGGL(vec_norms_kernel, dim3((unsigned)p), dim3(256), 0, s, t1, n, res_.as<double>());
      std::vector<double> rn(p), bn(p);
      CBFM_HIP(hipMemcpyAsync(rn.data(), res_.p, p * sizeof(double), hipMemcpyDeviceToHost, s));
      CBFM_HIP(hipMemcpyAsync(bn.data(), bnorm_.p, p * sizeof(double), hipMemcpyDeviceToHost, s));
      CBFM_HIP(hipStreamSynchronize(s));
      bool ok = true;
      for (int c = 0; c < p; ++c) {
        res[c] = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
        ok = ok && res[c] <= tol;
      }
      ++cycle;
      if (ok || total >= max_iter || K == 0) {
        noconv = !ok;
        return;
      }
    }
  }

 private:
  static uint64_t seed(int cycle, int64_t J, int pass) {
    return ((uint64_t)cycle * 65536 + (uint64_t)J) * 2 + (uint64_t)pass + 1;
  }
  // Out = the orthonormalised rows of W: Gram in double-double, pivoted
  // Cholesky, random rows past the rank
  void orthonormalise(const double2* W, double2* Out, double2* M, uint64_t sd, bool must_full) {
    const int32_t* ctl = ctl_.as<int32_t>();
    if (must_full)  // the second pass: rows already nearly orthonormal
      hipLaunchKernelGGL(gram_partial_kernel<false>, dim3((unsigned)nch_), dim3(256), 0, s_, W, n_, p_,
                         part_.as<double>(), ctl);
    else
      hipLaunchKernelGGL(gram_partial_kernel<true>, dim3((unsigned)nch_), dim3(256), 0, s_, W, n_, p_,
                         part_.as<double>(), ctl);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((p_ * p_ + 3) / 4)), dim3(256), 0, s_, part_.as<double>(),
                       nch_, p_, gdd_.as<double>(), ctl);
    hipLaunchKernelGGL(chol_pivot_kernel, dim3(1), dim3(256), 0, s_, gdd_.as<double>(), p_, 1e-26, M,
                       T_.as<double2>(), rank_.as<int32_t>(), ctl_.as<int32_t>(), must_full ? 1 : 0);
    hipLaunchKernelGGL(ortho_apply_kernel, dim3((unsigned)((n_ + 255) / 256), (unsigned)((p_ + 7) / 8)), dim3(256), 0,
                       s_, W, Out, n_, p_, T_.as<double2>(), rank_.as<int32_t>(), sd, ctl);
    CBFM_HIP(hipGetLastError());
  }
  // Iteration J on the main stream (the product, both projection and
  // orthonormalisation passes: the next basis block), and its block column
  // of the least-squares problem on the second stream, where it overlaps
  // iteration J + 1.  The passes' coefficients (C1, C2, M1, M2) alternate
  // between two buffers by the parity of J; iteration J + 2 waits until
  // the column kernel of iteration J has read them.
  void iteration(int64_t J, int cycle) {
    const int p = p_;
    const int64_t n = n_;
    const int par = (int)(J & 1);
    double2* V = V_.as<double2>();
    if (J >= 2) CBFM_HIP(hipStreamWaitEvent(s_, ev_read_[par], 0));
    if (mv_)
      mv_->launch((size_t)J, s_);
    else
      mvx_->launch((size_t)J, s_);
    const double vb = 16.0 * (double)(J + 1) * p * (double)n;  // bytes of the basis read by a pass
    for (int ps = 0; ps < 2; ++ps) {
      {
        TimedLaunch tl(T_GMRES_DOTS, s_, vb + 16.0 * p * (double)n);
        const size_t di = (size_t)(2 * J + ps);
        panel_batch(dots_dev_->as<GemmDesc>() + di, dots_[di], 1, 0, 0, 0, dots_ws_->as<double>(), s_);
      }
      {
        TimedLaunch tl(T_GMRES_UPDATE, s_, vb + 32.0 * p * (double)n);
        upd_->launch((size_t)(2 * J + ps), s_);
      }
      if (ps == 0)
        orthonormalise(t1_.as<double2>(), t2_.as<double2>(), M1(par), seed(cycle, J + 1, 0), false);
      else
        orthonormalise(t2_.as<double2>(), V + (J + 1) * p * n, M2(par), seed(cycle, J + 1, 1), true);
    }
    CBFM_HIP(hipEventRecord(ev_ready_[par], s_));
    CBFM_HIP(hipStreamWaitEvent(ls_, ev_ready_[par], 0));
    hipLaunchKernelGGL(bls_column_kernel, dim3((unsigned)p), dim3(256), 0, ls_, C1(par), C2(par), M1(par), M2(par),
                       Om_.as<double2>(), J, p, h_.as<double2>(), (mb_ + 2) * p, Rb_.as<double2>(), mb_ * p,
                       X_.as<double2>(), ctl_.as<int32_t>());
    CBFM_HIP(hipEventRecord(ev_read_[par], ls_));
    hipLaunchKernelGGL(bls_qr_kernel, dim3(1), dim3(256), 0, ls_, X_.as<double2>(), J, p, Rb_.as<double2>(), mb_ * p,
                       Om_.as<double2>(), G_.as<double2>(), bnorm_.as<double>(), tol_, res_.as<double>(),
                       ctl_.as<int32_t>());
    CBFM_HIP(hipGetLastError());
  }
  double2* C1(int par) const { return C1_.as<double2>() + (size_t)par * (mb_ + 1) * p_ * p_; }
  double2* C2(int par) const { return C2_.as<double2>() + (size_t)par * (mb_ + 1) * p_ * p_; }
  double2* M1(int par) const { return M1_.as<double2>() + (size_t)par * p_ * p_; }
  double2* M2(int par) const { return M2_.as<double2>() + (size_t)par * p_ * p_; }

 public:
  double tol_ = 1e-6;

 private:
  const double2* A_;
  int64_t lda_;
  const float2* A32_;
  int64_t lda32_, n_;
  int p_;
  int64_t mb_;
  hipStream_t s_;
  int nch_;
  Scratch V_, C1_, C2_, M1_, M2_, T_, rank_, part_, gdd_, G_, Rb_, Om_, h_, X_, Y_, bnorm_, res_, ctl_, t1_, t2_;
  std::vector<GemmDesc> dots_;
  std::unique_ptr<Scratch> dots_dev_, dots_ws_;
  std::unique_ptr<GemmPlan> mv_, upd_;
  std::unique_ptr<XGemmPlan> mvx_;
  hipStream_t ls_ = nullptr;  // the least-squares stream (default priority)
  hipEvent_t ev_ready_[2] = {nullptr, nullptr}, ev_read_[2] = {nullptr, nullptr};
};

}  // namespace

GmresResult block_gmres_run(const double2* A, int64_t lda, const float2* A32, int64_t lda32, int64_t n, int64_t nrhs,
                            const double2* b, double2* x, const GmresSpec& sp, hipStream_t s) {
  CBFM_REQUIRE(A != nullptr || A32 != nullptr, CBFM_E_ARG, "block GMRES needs a dense operator");
  CBFM_REQUIRE(n >= 2, CBFM_E_ARG, "block GMRES needs vectors of length 2 or more");
  CBFM_REQUIRE(sp.tol > 0 && sp.max_iter >= 1 && sp.restart >= 1, CBFM_E_ARG, "bad solver parameters");
  GmresResult out;
  out.its.assign(nrhs, 0);
  out.res.assign(nrhs, 1.0);
  // groups of sp.block right-hand sides (2..32), or with sp.block == 1 of
  // up to 32 with room for at least 32 block iterations per cycle
  // (restarted block GMRES with shorter cycles stagnates); at most n / 2,
  // so that a cycle holds at least one block iteration
  const int64_t want = sp.block >= 2 ? sp.block : std::max<int64_t>(1, n / 33);
  const int pg = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)PMAX, want, nrhs, n / 2}));
  for (int64_t g0 = 0; g0 < nrhs; g0 += pg) {
    const int p = (int)std::min<int64_t>(pg, nrhs - g0);
    // block iterations per cycle: the restart length, (mb + 1) p <= n, and
    // mb p <= RBUF (a block column of the triangular factor staged in LDS)
    const int64_t mb = std::max<int64_t>(1, std::min<int64_t>({sp.restart, n / p - 1, (int64_t)RBUF / p}));
    BlockGmres bg(A, lda, A32, lda32, n, p, mb, s);
    bg.tol_ = sp.tol;
    int64_t total = 0;
    std::vector<double> res(p, 1.0);
    bool noconv = false;
    bg.solve(b + g0 * n, x + g0 * n, sp.tol, sp.max_iter, total, res, noconv);
    for (int c = 0; c < p; ++c) {
      out.its[g0 + c] = (int32_t)total;
      out.res[g0 + c] = res[c];
    }
    out.noconv = out.noconv || noconv;
  }
  return out;
}

}  // namespace cbfm
