// Characteristic basis functions with dual orthogonalisation (paper Sec.
// III-A, III-B) and the Calderon preconditioner G^CBF (Sec. III-C).
//
// build:  per cell m
//   Z_mm   = cell block of [[K, -TE], [TH, K]]            (fill kernels, FP64)
//   J_m    = Z_mm^{-1} V_m  for the generating waves      (batched LU)
//   G'_m   = (J^M)^H G_m J^J, G_m the rotated RWG Gram
//   G'_m   = U S V^H, keep sigma_i / sigma_1 >= delta_svd
//   C^M_m  = J^M U_L,  C^J_m = J^J V_L
// The SVD is taken of an r x r core, r = min(s, N_m): with the QR
// factorisations (J^M)^H = Q_M R_M and (J^J)^H = Q_J R_J (Householder, R
// only), G'_m = Q_M X Q_J^H with X = R_M G_m R_J^H, so with X = U_c S V_c^H
// the singular values are those of G'_m and, since J^M Q_M = R_M^H,
// C^M_m = R_M^H U_c,L and C^J_m = R_J^H V_c,L (matrix-core GEMMs).  The
// core's SVD is one-sided Jacobi (one block per cell) on R_X^H, X = Q_X R_X,
// which yields S and V_c; U_c = X V_c S^{-1}.
// G_m is taken in closed form: for two RWGs a != b of one triangle with
// counter-clockwise local indices, int (n x f_a) . f_b = e_ab l_a l_b / 6
// times the RWG signs, e_ab = +1 if b follows a cyclically, -1 otherwise;
// it is zero on the diagonal and for RWGs sharing no triangle.
//
// G^CBF = blkdiag(A, B) with B = (C^M)^H G C^J and A = (C^J)^H G C^M =
// -B^H (G real antisymmetric), so one inverse of B serves both halves.

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <mutex>

#include "cbf.h"
#include "gemm.h"
#include "gj.h"
#include "solve.h"

namespace cbfm {

// ------------------------------------------------------------- kernels
// Gram entry G[e, f] of two canonical edges (closed form above).
__device__ double gram_entry(int e, int f, const int32_t* tplus, const int32_t* tminus, const int32_t* aplus,
                             const int32_t* aminus, const int32_t* tri_edge, const int32_t* tri_sign,
                             const double* length) {
  if (e == f) return 0.0;
  double g = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int t = side ? tminus[e] : tplus[e];
    const int a = side ? aminus[e] : aplus[e];
    for (int db = 1; db <= 2; ++db) {
      const int b = (a + db) % 3;
      if (tri_edge[t * 3 + b] == f) {
        const double eps = db == 1 ? 1.0 : -1.0;
        g += eps * length[e] * length[f] / 6.0 * tri_sign[t * 3 + a] * tri_sign[t * 3 + b];
      }
    }
  }
  return g;
}

// One cell of the batched per-cell launches: where its triangle-local blocks
// start in the local buffer of its group, and its support.
struct CellJob {
  int64_t loff;          // elements into the local buffer of the cell's group
  int32_t nt, N;         // support triangles, RWGs of the cell
  const int32_t* edges;  // the cell's RWGs (canonical edges)
  const int32_t* pos;    // mesh triangle -> position in the cell's support list
};

// Dense cell Grams G_m (N x N complex, row-major, cell b at b Nmax^2) of
// every cell's RWGs (blockIdx.z = cell).
__global__ void cell_gram_kernel(const CellJob* __restrict__ cells, int Nmax, const int32_t* tplus,
                                 const int32_t* tminus, const int32_t* aplus, const int32_t* aminus,
                                 const int32_t* tri_edge, const int32_t* tri_sign, const double* length,
                                 double2* __restrict__ G) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y, b = blockIdx.z;
  const CellJob cj = cells[b];
  if (c >= cj.N || r >= cj.N) return;
  G[(int64_t)b * Nmax * Nmax + (int64_t)r * cj.N + c] = make_double2(
      gram_entry(cj.edges[r], cj.edges[c], tplus, tminus, aplus, aminus, tri_edge, tri_sign, length), 0.0);
}

// Self blocks of a group of cells (blockIdx.z: cell cell0 + z): the cell's
// [[K, -TE], [TH, K]] as the first n columns of the row-major n x ld
// augmented system [Z_mm | V_m], with identity padding, each RWG entry the
// sum over the two triangles of either RWG of the triangle-local entries
// (local blocks [K, TE, TH], each 3 nt x 3 nt row-major; signs and lengths
// are inside them).
__global__ void cell_zmm_kernel(const double2* __restrict__ local, const CellJob* __restrict__ jobs, int cell0,
                                const int32_t* __restrict__ tplus, const int32_t* __restrict__ tminus,
                                const int32_t* __restrict__ aplus, const int32_t* __restrict__ aminus, int n,
                                int ld, double2* __restrict__ Aug) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= n) return;
  const int b = cell0 + (int)blockIdx.z;
  const CellJob jb = jobs[b];
  const int N = jb.N;
  double2 v = make_double2(r == c ? 1.0 : 0.0, 0.0);
  if (r < 2 * N && c < 2 * N) {
    const int br = r / N, bc = c / N, rr = r % N, cc = c % N;
    const int op = (br == bc) ? 0 : (br == 0 ? 1 : 2);
    const int64_t ldl = 3 * (int64_t)jb.nt, op_stride = ldl * ldl;
    const int32_t em = jb.edges[rr], en = jb.edges[cc];
    const int64_t ri[2] = {3 * (int64_t)jb.pos[tplus[em]] + aplus[em], 3 * (int64_t)jb.pos[tminus[em]] + aminus[em]};
    const int64_t ci[2] = {3 * (int64_t)jb.pos[tplus[en]] + aplus[en], 3 * (int64_t)jb.pos[tminus[en]] + aminus[en]};
    const double2* L = local + jb.loff + op * op_stride;
    double re = 0, im = 0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const double2 e = L[ri[x] * ldl + ci[y]];
        re += e.x;
        im += e.y;
      }
    v = (br == 0 && bc == 1) ? make_double2(-re, -im) : make_double2(re, im);
  }
  Aug[(int64_t)b * n * ld + (int64_t)r * ld + c] = v;
}

// The generating right-hand sides of every cell (blockIdx.z: cell): column
// n + c of the cell's row-major n x (n + S) augmented system is
// [v^E(edges); v^H(edges); 0] of wave c.
__global__ void cell_v_kernel(const double2* __restrict__ v, int64_t ne, const CellJob* __restrict__ jobs, int n,
                              int S, double2* __restrict__ Aug) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y, b = blockIdx.z;
  if (c >= S) return;
  const CellJob jb = jobs[b];
  double2 x = make_double2(0.0, 0.0);
  if (r < jb.N)
    x = v[(int64_t)c * 2 * ne + jb.edges[r]];
  else if (r < 2 * jb.N)
    x = v[(int64_t)c * 2 * ne + ne + jb.edges[r - jb.N]];
  Aug[((int64_t)b * n + r) * (n + S) + n + c] = x;
}

// From every cell's solved currents J = [J^M; J^J] (columns n .. n + S - 1
// of the row-major n x (n + S) augmented system, the magnetic rows first), write (J^M)^H and (J^J)^H as column-major
// S x Nmax matrices (blockIdx.z = 2 cell + which), zero beyond the cell's N
// columns.
__global__ void pack_jh_kernel(const double2* __restrict__ J, int n, int S, const int32_t* __restrict__ Ns, int Nmax,
                               double2* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y, b = blockIdx.z >> 1, w = blockIdx.z & 1;
  if (r >= S) return;
  const int N = Ns[b];
  double2 x = make_double2(0.0, 0.0);
  if (c < N) {
    x = J[((int64_t)b * n + w * N + c) * (n + S) + n + r];
    x.y = -x.y;
  }
  out[((int64_t)(2 * b + w) * Nmax + c) * S + r] = x;
}

__device__ inline double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// In-place Householder QR of the column-major m x ncol matrix A (lda), only R
// kept: afterwards the upper triangle of the first kmax = min(m, ncol) rows
// holds R and the entries below the diagonal of the first kmax columns are
// zero.  Reflector k is H = I - beta v v^H with v = x - alpha e_1, x the
// column below the diagonal, alpha = -e^{i arg x_0} ||x||, beta = 2 / v^H v =
// 1 / (||x||^2 + |x_0| ||x||).  Every thread of the block calls it; v is LDS
// scratch of m entries, sc one LDS double.
template <typename P>
__device__ void householder_r(P A, int lda, int m, int ncol, double2* v, double* sc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int kmax = min(m, ncol);
  for (int k = 0; k < kmax; ++k) {
    P col = A + (int64_t)k * lda;
    if (wave == 0) {
      double q = 0;
      for (int i = k + lane; i < m; i += 64) {
        const double2 x = col[i];
        q += x.x * x.x + x.y * x.y;
      }
      q = wave_sum(q);
      const double nx = sqrt(q);
      const double2 x0 = col[k];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double2 ph = ax0 > 0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 alpha = make_double2(-ph.x * nx, -ph.y * nx);
      for (int i = k + lane; i < m; i += 64) {
        double2 x = col[i];
        if (i == k) x = make_double2(x.x - alpha.x, x.y - alpha.y);
        v[i] = x;
        col[i] = i == k ? alpha : make_double2(0.0, 0.0);
      }
      if (lane == 0) *sc = nx > 0 ? 1.0 / (q + ax0 * nx) : 0.0;
    }
    __syncthreads();
    const double beta = *sc;
    if (beta != 0.0) {
      for (int j = k + 1 + wave; j < ncol; j += nw) {
        P cj = A + (int64_t)j * lda;
        double wr = 0, wi = 0;  // v^H a
        for (int i = k + lane; i < m; i += 64) {
          const double2 a = cj[i], w = v[i];
          wr += w.x * a.x + w.y * a.y;
          wi += w.x * a.y - w.y * a.x;
        }
        wr = beta * wave_sum(wr);
        wi = beta * wave_sum(wi);
        for (int i = k + lane; i < m; i += 64) {
          const double2 w = v[i];
          double2 a = cj[i];
          a.x -= wr * w.x - wi * w.y;
          a.y -= wr * w.y + wi * w.x;
          cj[i] = a;
        }
      }
    }
    __syncthreads();
  }
}

// R factors of (J^M)^H and (J^J)^H of every cell: block b takes the column-
// major S x Nmax matrix b of qa (cell b / 2, its first N columns) and writes
// R as row-major rk x Nmax (zero below the diagonal and beyond column N).
__global__ void __launch_bounds__(1024) cell_qr_kernel(double2* __restrict__ qa, int S, int Nmax,
                                                       const int32_t* __restrict__ ncell, int rk,
                                                       double2* __restrict__ R) {
  extern __shared__ double2 v[];  // S entries
  __shared__ double sc;
  const int b = blockIdx.x, N = ncell[b / 2];
  double2* A = qa + (int64_t)b * S * Nmax;
  householder_r(A, S, S, N, v, &sc);
  const int kmax = min(S, N);
  double2* Rb = R + (int64_t)b * rk * Nmax;
  for (int64_t e = threadIdx.x; e < (int64_t)rk * Nmax; e += blockDim.x) {
    const int i = (int)(e / Nmax), j = (int)(e % Nmax);
    Rb[e] = (i <= j && j < N && i < kmax) ? A[(int64_t)j * S + i] : make_double2(0.0, 0.0);
  }
}

// x moved across the lanes of each row of 16 by a DPP pattern.
template <int CTRL>
__device__ inline double dpp_double(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes; a butterfly, so every lane of the row ends
// with the same bits.
__device__ inline double row16_sum(double x) {
  x += dpp_double<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_double<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_double<0x141>(x);  // row_half_mirror: the other quad of the half row
  x += dpp_double<0x140>(x);  // row_mirror: the other half row
  return x;
}

// One-sided (Hestenes) Jacobi on the columns of the column-major nc x nc
// matrix B (ldb): pairs of columns are rotated, in the round-robin order that
// lets each row of 16 lanes of the block rotate a disjoint pair at once, until
// in one sweep no pair has |b_p^H b_q| > tol ||b_p|| ||b_q||.  The 2 x 2 step
// for alpha = ||b_p||^2, beta = ||b_q||^2, gamma = b_p^H b_q = |gamma| e:
// zeta = (beta - alpha) / (2 |gamma|), t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t,
// (b_p, b_q) <- (c b_p - s conj(e) b_q, s e b_p + c b_q).
// Returns the number of sweeps, or -1 if max_sweeps ran out.
template <typename P>
__device__ int hestenes_jacobi(P B, int ldb, int nc, double tol, int max_sweeps, int* flag) {
  const int gl = threadIdx.x & 15, grp = threadIdx.x >> 4, ngrp = blockDim.x >> 4;
  const int ne = nc + (nc & 1);  // an odd count plays against an empty column
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int step = 0; step < ne - 1; ++step) {
      for (int pr = grp; pr < ne / 2; pr += ngrp) {
        const int qr = ne - 1 - pr;
        const int p = pr == 0 ? 0 : 1 + (pr - 1 + step) % (ne - 1);
        const int q = 1 + (qr - 1 + step) % (ne - 1);
        if (p >= nc || q >= nc) continue;
        P x = B + (int64_t)p * ldb;
        P y = B + (int64_t)q * ldb;
        double al = 0, be = 0, gr = 0, gi = 0;
        for (int i = gl; i < nc; i += 16) {
          const double2 a = x[i], c = y[i];
          al += a.x * a.x + a.y * a.y;
          be += c.x * c.x + c.y * c.y;
          gr += a.x * c.x + a.y * c.y;
          gi += a.x * c.y - a.y * c.x;
        }
        al = row16_sum(al);
        be = row16_sum(be);
        gr = row16_sum(gr);
        gi = row16_sum(gi);
        const double ag = sqrt(gr * gr + gi * gi);
        if (!(al * be > 0 && ag > tol * sqrt(al * be))) continue;  // same on the 16 lanes
        const double z = (be - al) / (2.0 * ag);
        const double t = (z >= 0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        const double er = gr / ag, ei = gi / ag;
        for (int i = gl; i < nc; i += 16) {
          const double2 a = x[i], c = y[i];
          // a' = cs a - sn conj(e) c ;  c' = sn e a + cs c
          x[i] = make_double2(cs * a.x - sn * (er * c.x + ei * c.y), cs * a.y - sn * (er * c.y - ei * c.x));
          y[i] = make_double2(sn * (er * a.x - ei * a.y) + cs * c.x, sn * (er * a.y + ei * a.x) + cs * c.y);
        }
        if (gl == 0) *flag = 1;
      }
      __syncthreads();
    }
    if (*flag == 0) return sweep + 1;
  }
  return -1;
}

// SVD of each cell's core X (column-major rk x rk, leading nc = min(N, rk)
// block nonzero): X = Q R (Householder), then one-sided Jacobi on B = R^H,
// B W = U~ S.  Since R = W S U~^H, X = (Q W) S U~^H: U~ are the right
// singular vectors of X and S its singular values.  Written sorted by
// decreasing sigma: sigma (rk per cell, zero beyond nc), Ut = U~ and
// Uts = U~ S^{-1} (column-major rk x rk, first nc columns, zero rows beyond
// nc), info = 0, or 1 if the sweeps ran out.  LDS = true keeps the nc x nc
// working matrix in LDS, else in work (rk x rk per cell).
template <bool LDS>
__global__ void __launch_bounds__(1024) core_svd_kernel(const double2* __restrict__ X, int rk,
                                                        const int32_t* __restrict__ ncell, double2* work, double tol,
                                                        int max_sweeps, double* __restrict__ sigma,
                                                        double2* __restrict__ Ut, double2* __restrict__ Uts,
                                                        int32_t* __restrict__ info) {
  extern __shared__ double2 lds[];
  __shared__ double sc;
  __shared__ int flag;
  const int b = blockIdx.x, nc = min((int)ncell[b], rk);
  double2* A = LDS ? lds : work + (int64_t)b * rk * rk;
  double2* v = LDS ? lds + (int64_t)nc * nc : lds;            // nc entries
  double* nrm = reinterpret_cast<double*>(v + nc);             // nc entries
  int* rank = reinterpret_cast<int*>(nrm + nc);                // nc entries
  const double2* Xb = X + (int64_t)b * rk * rk;
  for (int64_t e = threadIdx.x; e < (int64_t)nc * nc; e += blockDim.x) {
    const int i = (int)(e % nc), j = (int)(e / nc);
    A[e] = Xb[(int64_t)j * rk + i];
  }
  __syncthreads();
  householder_r(A, nc, nc, nc, v, &sc);
  // B = R^H in place (lower triangular)
  for (int64_t e = threadIdx.x; e < (int64_t)nc * nc; e += blockDim.x) {
    const int i = (int)(e % nc), j = (int)(e / nc);
    if (i < j) continue;
    const double2 r = A[(int64_t)i * nc + j];  // R[j][i]
    A[e] = make_double2(r.x, -r.y);
    if (i > j) A[(int64_t)i * nc + j] = make_double2(0.0, 0.0);
  }
  const int sweeps = hestenes_jacobi(A, nc, nc, tol, max_sweeps, &flag);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = wave; j < nc; j += nw) {
    double q = 0;
    for (int i = lane; i < nc; i += 64) {
      const double2 a = A[(int64_t)j * nc + i];
      q += a.x * a.x + a.y * a.y;
    }
    q = wave_sum(q);
    if (lane == 0) nrm[j] = sqrt(q);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nc; j += blockDim.x) {
    int r = 0;
    for (int k = 0; k < nc; ++k) r += (nrm[k] > nrm[j] || (nrm[k] == nrm[j] && k < j)) ? 1 : 0;
    rank[j] = r;
    sigma[(int64_t)b * rk + r] = nrm[j];
  }
  for (int j = nc + (int)threadIdx.x; j < rk; j += blockDim.x) sigma[(int64_t)b * rk + j] = 0.0;
  __syncthreads();
  for (int j = wave; j < nc; j += nw) {
    const double sg = nrm[j];
    const double s1 = sg > 0 ? 1.0 / sg : 0.0, s2 = s1 * s1;
    double2* u = Ut + (int64_t)b * rk * rk + (int64_t)rank[j] * rk;
    double2* us = Uts + (int64_t)b * rk * rk + (int64_t)rank[j] * rk;
    for (int i = lane; i < rk; i += 64) {
      const double2 a = i < nc ? A[(int64_t)j * nc + i] : make_double2(0.0, 0.0);
      u[i] = make_double2(a.x * s1, a.y * s1);
      us[i] = make_double2(a.x * s2, a.y * s2);
    }
  }
  if (threadIdx.x == 0) info[b] = sweeps < 0 ? 1 : 0;
}

// GC[m][col] = sum_n G[perm[m], n] C^J_full[n][col], rows in internal order.
__global__ void gram_times_cj_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
                                     const int32_t* __restrict__ edge_block, const int64_t* __restrict__ cell_off,
                                     const int64_t* __restrict__ off, const int32_t* __restrict__ L,
                                     const int64_t* __restrict__ coff, const double2* __restrict__ CJ, int64_t ne,
                                     int64_t NL, const int32_t* tplus, const int32_t* tminus, const int32_t* aplus,
                                     const int32_t* aminus, const int32_t* tri_edge, const int32_t* tri_sign,
                                     const double* length, double2* __restrict__ GC) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, m = blockIdx.y;
  if (col >= NL) return;
  const int e = perm[m];
  double2 acc = make_double2(0.0, 0.0);
  for (int side = 0; side < 2; ++side) {
    const int t = side ? tminus[e] : tplus[e];
    const int a = side ? aminus[e] : aplus[e];
    for (int db = 1; db <= 2; ++db) {
      const int b = (a + db) % 3;
      const int f = tri_edge[t * 3 + b];
      const double g = (db == 1 ? 1.0 : -1.0) * length[e] * length[f] / 6.0 * tri_sign[t * 3 + a] * tri_sign[t * 3 + b];
      const int cf = edge_block[f];
      if (col >= off[cf] && col < off[cf] + L[cf]) {
        const int64_t row = iperm[f] - cell_off[cf];
        const double2 c = CJ[coff[cf] + row * L[cf] + (col - off[cf])];
        acc.x += g * c.x;
        acc.y += g * c.y;
      }
    }
  }
  GC[m * NL + col] = acc;
}

// The same product for a block-diagonal B, kept per cell: GCc at coff[a]
// holds G_aa C^J_a (N_a x L_a row-major; no RWG's Gram row reaches another
// cell).  One block per RWG row m (internal order), lanes over its cell's
// columns.
__global__ void gram_times_cj_cell_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
                                          const int32_t* __restrict__ edge_block, const int64_t* __restrict__ cell_off,
                                          const int32_t* __restrict__ L, const int64_t* __restrict__ coff,
                                          const double2* __restrict__ CJ, int64_t ne, const int32_t* tplus,
                                          const int32_t* tminus, const int32_t* aplus, const int32_t* aminus,
                                          const int32_t* tri_edge, const int32_t* tri_sign, const double* length,
                                          double2* __restrict__ GCc) {
  const int64_t m = blockIdx.x;
  if (m >= ne) return;
  const int e = perm[m], a = edge_block[e], La = L[a];
  const int64_t r = m - cell_off[a];
  for (int j = threadIdx.x; j < La; j += blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int side = 0; side < 2; ++side) {
      const int t = side ? tminus[e] : tplus[e];
      const int ai = side ? aminus[e] : aplus[e];
      for (int db = 1; db <= 2; ++db) {
        const int b = (ai + db) % 3;
        const int f = tri_edge[t * 3 + b];
        const double g = (db == 1 ? 1.0 : -1.0) * length[e] * length[f] / 6.0 * tri_sign[t * 3 + ai] * tri_sign[t * 3 + b];
        const double2 c = CJ[coff[a] + (iperm[f] - cell_off[a]) * La + j];
        acc.x += g * c.x;
        acc.y += g * c.y;
      }
    }
    GCc[coff[a] + r * La + j] = acc;
  }
}

// ------------------------------------------------------------- host helpers
static std::vector<int32_t> cell_edges(const MeshHost& h, int b) {
  return std::vector<int32_t>(h.perm.begin() + h.cell_off[b], h.perm.begin() + h.cell_off[b + 1]);
}

void cbf_finish(cbfm_cbf_s* c) {
  const MeshHost& h = c->mesh->h;
  c->off.assign(h.nblocks + 1, 0);
  c->coff.assign(h.nblocks + 1, 0);
  for (int b = 0; b < h.nblocks; ++b) {
    c->off[b + 1] = c->off[b] + c->L[b];
    c->coff[b + 1] = c->coff[b] + (h.cell_off[b + 1] - h.cell_off[b]) * (int64_t)c->L[b];
  }
  c->NL = c->off[h.nblocks];
  std::vector<int32_t> tcell(h.nt, -1);
  c->blockdiag = true;
  for (int64_t e = 0; e < h.ne && c->blockdiag; ++e)
    for (const int32_t t : {h.tplus[e], h.tminus[e]}) {
      if (tcell[t] < 0)
        tcell[t] = h.edge_block[e];
      else if (tcell[t] != h.edge_block[e])
        c->blockdiag = false;
    }
  c->d_L.upload(c->L);
  c->d_off.upload(c->off);
  c->d_coff.upload(c->coff);
  c->d_cell_off.upload(h.cell_off);
  c->d_edge_block.upload(h.edge_block);
}

// Diagonal blocks of a block-diagonal B (row-major NL x NL, cell a at rows
// and columns off[a] .. off[a] + L[a]) to or from a stack of Lmax x Lmax
// row-major blocks padded with the identity (blockIdx.z = cell).
__global__ void cmp_blocks_kernel(double2* __restrict__ B, int64_t NL, const int64_t* __restrict__ off,
                                  const int32_t* __restrict__ L, int Lmax, double2* __restrict__ P, int to_stack) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y, a = blockIdx.z;
  if (j >= Lmax) return;
  const int La = L[a];
  double2* p = P + ((int64_t)a * Lmax + i) * Lmax + j;
  const bool in = i < La && j < La;
  double2* b = B + (off[a] + (in ? i : 0)) * NL + off[a] + (in ? j : 0);
  if (to_stack)
    *p = in ? *b : make_double2(i == j ? 1.0 : 0.0, 0.0);
  else if (in)
    *b = *p;
}

// Invert the diagonal blocks of a block-diagonal B in place (one batched
// Gauss-Jordan inversion, blocks padded with the identity to the largest);
// the blocks off the diagonal are zeros and stay so.  async: the pivot
// checks are left in c->dinfo, nothing is waited for.
static void invert_blocks(cbfm_cbf_s* c, hipStream_t s, bool async) {
  const MeshHost& h = c->mesh->h;
  const int64_t NL = c->NL;
  const int nb = h.nblocks;
  const int Lmax = *std::max_element(c->L.begin(), c->L.end());
  Scratch P((size_t)nb * Lmax * Lmax * sizeof(double2), s);
  const dim3 g((unsigned)((Lmax + 63) / 64), (unsigned)Lmax, (unsigned)nb);
  hipLaunchKernelGGL(cmp_blocks_kernel, g, dim3(64), 0, s, c->Binv.as<double2>(), NL, c->d_off.as<int64_t>(),
                     c->d_L.as<int32_t>(), Lmax, P.as<double2>(), 1);
  CBFM_HIP(hipGetLastError());
  if (async) {
    c->dinfo.alloc((size_t)nb * sizeof(int32_t));
    c->ninfo = nb;
    gj_inverse_batched_async(P.as<double2>(), (int64_t)Lmax * Lmax, Lmax, nb, c->dinfo.as<int32_t>(), s);
  } else {
    gj_inverse_batched(P.as<double2>(), (int64_t)Lmax * Lmax, Lmax, nb, "G^CBF block of cell", s);
  }
  hipLaunchKernelGGL(cmp_blocks_kernel, g, dim3(64), 0, s, c->Binv.as<double2>(), NL, c->d_off.as<int64_t>(),
                     c->d_L.as<int32_t>(), Lmax, P.as<double2>(), 0);
  CBFM_HIP(hipGetLastError());
}

// B^{-1} for B = (C^M)^H G C^J (row-major, inverted in place by blocked
// Gauss-Jordan elimination).  A block-diagonal B is inverted block by block
// (one batched call; the blocks off the diagonal are exact zeros and stay
// so).  async: enqueue only, the pivot checks left in c->dinfo (the caller
// marks the result pending); else checked, and c->factored set.
// B = (C^M)^H G C^J (NL x NL row-major) into Bout: cell by cell when no
// triangle carries RWGs of two cells (the blocks off the diagonal are then
// exact zeros), else through the RWG Gram times C^J of every cell.
static void form_b(cbfm_cbf_s* c, double2* Bout, hipStream_t s) {
  const cbfm_mesh_s* m = c->mesh;
  const MeshHost& h = m->h;
  const int64_t NL = c->NL, ne = h.ne;
  if (c->blockdiag) {
    // B_a = (C^M_a)^H G_aa C^J_a per cell into the zeroed B
    const int nb = h.nblocks;
    Scratch GCc((size_t)std::max<int64_t>(1, c->coff[nb]) * sizeof(double2), s);
    hipLaunchKernelGGL(gram_times_cj_cell_kernel, dim3((unsigned)ne), dim3(64), 0, s, m->perm.as<int32_t>(),
                       m->iperm.as<int32_t>(), c->d_edge_block.as<int32_t>(), c->d_cell_off.as<int64_t>(),
                       c->d_L.as<int32_t>(), c->d_coff.as<int64_t>(), c->CJ.as<double2>(), ne, m->tplus.as<int32_t>(),
                       m->tminus.as<int32_t>(), m->aplus.as<int32_t>(), m->aminus.as<int32_t>(),
                       m->tri_edge.as<int32_t>(), m->tri_sign.as<int32_t>(), m->length.as<double>(), GCc.as<double2>());
    CBFM_HIP(hipGetLastError());
    CBFM_HIP(hipMemsetAsync(Bout, 0, NL * NL * sizeof(double2), s));
    std::vector<GemmDesc> ds;
    for (int a = 0; a < nb; ++a) {
      const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], La = c->L[a];
      ds.push_back(gemm(c->CM.as<double2>() + c->coff[a], La, OP_C, GCc.as<double2>() + c->coff[a], La, OP_N,
                        Bout + c->off[a] * NL + c->off[a], NL, La, La, Na));
    }
    zgemm_batched(ds, s);
    return;
  }
  CBFM_REQUIRE(ne <= 65535, CBFM_E_ARG, "G^CBF coupling cells: at most 65535 RWGs");
  Scratch GC(ne * NL * sizeof(double2), s);
  dim3 grid((unsigned)((NL + 255) / 256), (unsigned)ne);
  hipLaunchKernelGGL(gram_times_cj_kernel, grid, dim3(256), 0, s, m->perm.as<int32_t>(), m->iperm.as<int32_t>(),
                     c->d_edge_block.as<int32_t>(), c->d_cell_off.as<int64_t>(), c->d_off.as<int64_t>(),
                     c->d_L.as<int32_t>(), c->d_coff.as<int64_t>(), c->CJ.as<double2>(), ne, NL,
                     m->tplus.as<int32_t>(), m->tminus.as<int32_t>(), m->aplus.as<int32_t>(), m->aminus.as<int32_t>(),
                     m->tri_edge.as<int32_t>(), m->tri_sign.as<int32_t>(), m->length.as<double>(), GC.as<double2>());
  CBFM_HIP(hipGetLastError());
  std::vector<GemmDesc> ds;
  for (int a = 0; a < h.nblocks; ++a) {
    const int64_t Na = h.cell_off[a + 1] - h.cell_off[a];
    ds.push_back(gemm(c->CM.as<double2>() + c->coff[a], c->L[a], OP_C, GC.as<double2>() + h.cell_off[a] * NL, NL,
                      OP_N, Bout + c->off[a] * NL, NL, c->L[a], NL, Na));
  }
  zgemm_batched(ds, s);
}

static void cmp_factor(cbfm_cbf_s* c, hipStream_t s, bool async = false) {
  const int64_t NL = c->NL;
  c->Binv.alloc(NL * NL * sizeof(double2));
  form_b(c, c->Binv.as<double2>(), s);
  if (c->blockdiag) {
    invert_blocks(c, s, async);
    if (!async) c->factored = true;
    return;
  }
  CBFM_REQUIRE(NL <= 65535, CBFM_E_ARG, "G^CBF coupling cells: at most 65535 CBFs per current");
  if (async) {
    c->dinfo.alloc(sizeof(int32_t));
    c->ninfo = 1;
    gj_inverse_batched_async(c->Binv.as<double2>(), NL * NL, (int)NL, 1, c->dinfo.as<int32_t>(), s);
    return;
  }
  gj_inverse_batched(c->Binv.as<double2>(), NL * NL, (int)NL, 1, "G^CBF", s);
  c->factored = true;
}

// The operator of the inexact CMP: Gd = G^CBF D^CBF (2NL x 2NL, row-major)
// with G^CBF = blkdiag(-B^H, B) and D^CBF = diag(1 / [G^CBF]_jj) (1 where
// that diagonal is 0), and D^CBF itself (row i = 0 writes it).
__global__ void inner_operator_kernel(const double2* __restrict__ B, int64_t NL, double2* __restrict__ Gd,
                                      double2* __restrict__ dinv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y, n = 2 * NL;
  if (j >= n) return;
  double2 g = make_double2(0.0, 0.0), dg;
  if (j < NL) {
    const double2 b = B[j * NL + j];
    dg = make_double2(-b.x, b.y);  // -conj(B_jj)
    if (i < NL) {
      const double2 e = B[j * NL + i];  // (-B^H)_ij = -conj(B_ji)
      g = make_double2(-e.x, e.y);
    }
  } else {
    dg = B[(j - NL) * NL + (j - NL)];
    if (i >= NL) g = B[(i - NL) * NL + (j - NL)];
  }
  const double den = dg.x * dg.x + dg.y * dg.y;
  const double2 d = den > 0 ? make_double2(dg.x / den, -dg.y / den) : make_double2(1.0, 0.0);
  Gd[i * n + j] = make_double2(g.x * d.x - g.y * d.y, g.x * d.y + g.y * d.x);
  if (i == 0) dinv[j] = d;
}

__global__ void diag_times_kernel(const double2* __restrict__ d, const double2* __restrict__ z, double2* __restrict__ x,
                                  int64_t n, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (i >= n || c >= nv) return;
  const double2 a = d[i], b = z[c * n + i];
  x[c * n + i] = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

void cmp_inner_apply(cbfm_cbf_s* c, int64_t nrhs, const double2* y, double2* x, double tol, hipStream_t s) {
  const int64_t NL = c->NL, n = 2 * NL;
  if (nrhs == 0 || NL == 0) return;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->inner_ready) {
      CBFM_REQUIRE(n <= 65535, CBFM_E_ARG, "inexact CMP: at most 32767 CBFs per current");
      Scratch B((size_t)NL * NL * sizeof(double2), s);
      form_b(c, B.as<double2>(), s);
      c->Gd.alloc((size_t)n * n * sizeof(double2));
      c->dinv.alloc((size_t)n * sizeof(double2));
      hipLaunchKernelGGL(inner_operator_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s,
                         B.as<double2>(), NL, c->Gd.as<double2>(), c->dinv.as<double2>());
      CBFM_HIP(hipGetLastError());
      c->inner_ready = true;
    }
  }
  // GMRES on (G^CBF D^CBF) z = y, x = D^CBF z
  GmresSpec sp;
  sp.tol = tol;
  sp.restart = std::min<int64_t>(n, 500);
  sp.max_iter = 4 * n;
  DenseOp op(c->Gd.as<double2>(), n, nullptr, 0);
  Scratch z((size_t)nrhs * n * sizeof(double2), s);
  (void)gmres_run(op, n, nrhs, y, z.as<double2>(), sp, s);
  hipLaunchKernelGGL(diag_times_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, s,
                     c->dinv.as<double2>(), z.as<double2>(), x, n, nrhs);
  CBFM_HIP(hipGetLastError());
}

// A side stream per device and host thread (default priority) for work that
// overlaps the caller's stream.  Non-blocking: a blocking stream would
// synchronise with the legacy default stream that callers often use, and the
// overlap would be lost; the ordering is explicit (events) both ways.
static hipStream_t side_stream() {
  static thread_local std::map<int, hipStream_t> streams;
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  auto it = streams.find(dev);
  if (it == streams.end()) {
    hipStream_t st = nullptr;
    CBFM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    scratch_side_stream(st);
    it = streams.emplace(dev, st).first;
  }
  return it->second;
}

static thread_local bool t_async_cmp = true;
void async_cmp_on_this_thread(bool on) { t_async_cmp = on; }

// Start B^{-1} on the side stream after the work queued so far on s (the
// CBF build), so that it overlaps what the caller queues next; the first
// cmp_inverse waits for it and checks its pivots.  On any failure here the
// handle is left unfactored and cmp_inverse forms B^{-1} itself.
static void cmp_factor_async(cbfm_cbf_s* c, hipStream_t s) {
  hipStream_t side = nullptr;
  try {
    side = side_stream();
    // (both events live as long as the handle: none is destroyed while a
    // wait on it may still be queued)
    if (!c->start) CBFM_HIP(hipEventCreateWithFlags(&c->start, hipEventDisableTiming));
    if (!c->done) CBFM_HIP(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
    CBFM_HIP(hipEventRecord(c->start, s));
    CBFM_HIP(hipStreamWaitEvent(side, c->start, 0));
    cmp_factor(c, side, true);
    CBFM_HIP(hipEventRecord(c->done, side));
    c->pending = true;
  } catch (...) {
    if (side) (void)hipStreamSynchronize(side);
    (void)hipGetLastError();
    c->pending = false;
    c->factored = false;
  }
}

const double2* cmp_inverse(cbfm_cbf_s* c, hipStream_t s) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->pending) {
    c->pending = false;
    CBFM_HIP(hipStreamWaitEvent(s, c->done, 0));
    gj_check(c->dinfo.as<int32_t>(), c->ninfo, c->blockdiag ? "G^CBF block of cell" : "G^CBF", s);
    c->factored = true;
  }
  if (!c->factored) cmp_factor(c, s);
  return c->Binv.as<double2>();
}

// x <- (G^CBF)^{-1} x with (G^CBF)^{-1} = blkdiag(-(B^{-1})^H, B^{-1}); for
// vectors stored as rows: x1 <- -x1 conj(B^{-1}),  x2 <- x2 (B^{-1})^T.
void cmp_apply_dev(cbfm_cbf_s* c, int64_t nrhs, double2* x, hipStream_t s) {
  const double2* Bi = cmp_inverse(c, s);
  const int64_t NL = c->NL, n = 2 * NL;
  if (nrhs == 0 || NL == 0) return;
  Scratch y(nrhs * n * sizeof(double2), s);
  CBFM_HIP(hipMemcpyAsync(y.p, x, nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  std::vector<GemmDesc> ds{gemm(y.as<double2>(), n, OP_N, Bi, NL, OP_R, x, n, nrhs, NL, NL, -1.0),
                           gemm(y.as<double2>() + NL, n, OP_N, Bi, NL, OP_T, x + NL, n, nrhs, NL, NL)};
  zgemm_batched(ds, s);
}

// Dynamic LDS that a core_svd_kernel<true> block may use on the current
// device (the kernel's attribute is raised to it once per device).
static size_t core_svd_lds_limit() {
  static std::mutex mu;
  static std::map<int, size_t> limit;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  auto it = limit.find(dev);
  if (it != limit.end()) return it->second;
  int maxsh = 0;
  CBFM_HIP(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  size_t lim = maxsh > 256 ? (size_t)maxsh - 256 : 0;  // room for the kernel's static LDS
  if (lim > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(&core_svd_kernel<true>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess) {
    (void)hipGetLastError();
    lim = 65536;
  }
  limit[dev] = lim;
  return lim;
}

// Per-cell support triangles and the near pairs inside it.
struct CellSupport {
  std::vector<int32_t> tris, pos, edges;
  std::vector<NearPair> near;
};

// The supports of all cells, with each cell's near pairs in the order of
// the mesh's near list (one pass over the list: a triangle lies in the
// supports of at most the three cells of its edges).
static std::vector<CellSupport> supports(const MeshHost& h, int nb) {
  std::vector<CellSupport> cs(nb);
  std::vector<std::array<int32_t, 3>> tcell(h.nt, {-1, -1, -1});
  for (int b = 0; b < nb; ++b) {
    CellSupport& c = cs[b];
    c.edges = cell_edges(h, b);
    c.pos.assign(h.nt, -1);
    for (int32_t e : c.edges) {
      c.pos[h.tplus[e]] = 0;
      c.pos[h.tminus[e]] = 0;
    }
    for (int64_t t = 0; t < h.nt; ++t)
      if (c.pos[t] == 0) {
        c.pos[t] = (int32_t)c.tris.size();
        c.tris.push_back((int32_t)t);
        for (int32_t& x : tcell[t])
          if (x < 0) {
            x = b;
            break;
          }
      }
  }
  for (const NearPair& q : h.near)
    for (int32_t b : tcell[q.p]) {
      if (b < 0) break;
      if (cs[b].pos[q.q] >= 0) cs[b].near.push_back({q.p, q.q, cs[b].pos[q.p], cs[b].pos[q.q], q.coplanar, 0});
    }
  return cs;
}

}  // namespace cbfm

using namespace cbfm;

cbfm_cbf_s::~cbfm_cbf_s() {
  if (done) {
    (void)hipEventSynchronize(done);
    (void)hipEventDestroy(done);
  }
  if (start) {
    (void)hipEventSynchronize(start);
    (void)hipEventDestroy(start);
  }
}

// CBFs of every cell from its current coefficient sets J_m = [J^M_m; J^J_m]
// (primary or IPCBF), given as (J^M_m)^H and (J^J_m)^H in QA: column-major
// S x Nmax per cell and current (cell b's at 2 b and 2 b + 1), zero beyond
// the cell's N_m columns.  The dual orthogonalisation of Sec. III-B: QR of
// both (R only), the core X = R_M G_m R_J^H, its one-sided Jacobi SVD,
// L_m = #{sigma_i / sigma_1 >= delta_svd} (at most max_L), C^M = J^M U_L,
// C^J = J^J V_L.  share: every cell takes cell 0's CBFs (arrays of
// translated copies).  The CMP inverse is queued on the side stream unless
// this thread disabled that.  Returns a new handle; QA is overwritten.
static cbfm_cbf_s* orthogonalise(const cbfm_mesh_s* m, double2* QA_p, int S, int Nmax, const std::vector<int32_t>& hN,
                                 const int32_t* dN_p, const CellJob* djobs, double delta_svd, int max_L, bool share,
                                 hipStream_t s) {
  const MeshHost& h = m->h;
  const int nb = h.nblocks;
  const int rk = std::min(S, Nmax);
  Scratch info((size_t)nb * sizeof(int32_t), s);  // per cell: the Jacobi SVD ran out of sweeps
  std::vector<int32_t> hinfo(nb);
  Scratch Rf((size_t)nb * 2 * rk * Nmax * sizeof(double2), s);  // per cell R_M, then R_J
  hipLaunchKernelGGL(cell_qr_kernel, dim3(2 * nb), dim3(1024), (size_t)S * sizeof(double2), s, QA_p, S,
                     Nmax, dN_p, rk, Rf.as<double2>());
  CBFM_HIP(hipGetLastError());
  // core X = R_M G_m R_J^H (column-major rk x rk), computed as its row-major
  // transpose conj(R_J) G_m^T R_M^T = -conj(R_J) G_m R_M^T (G_m antisymmetric)
  Scratch Gm((size_t)nb * Nmax * Nmax * sizeof(double2), s);
  Scratch T2((size_t)nb * Nmax * rk * sizeof(double2), s);
  Scratch core((size_t)nb * rk * rk * sizeof(double2), s);
  hipLaunchKernelGGL(cell_gram_kernel, dim3((Nmax + 255) / 256, Nmax, nb), dim3(256), 0, s, djobs, Nmax,
                     m->tplus.as<int32_t>(), m->tminus.as<int32_t>(), m->aplus.as<int32_t>(), m->aminus.as<int32_t>(),
                     m->tri_edge.as<int32_t>(), m->tri_sign.as<int32_t>(), m->length.as<double>(), Gm.as<double2>());
  std::vector<GemmDesc> d1, d2;
  for (int b = 0; b < nb; ++b) {
    const int Nb = hN[b];
    const double2* R = Rf.as<double2>() + (size_t)b * 2 * rk * Nmax;
    double2* G = Gm.as<double2>() + (size_t)b * Nmax * Nmax;
    double2* t2 = T2.as<double2>() + (size_t)b * Nmax * rk;
    d1.push_back(gemm(G, Nb, OP_N, R, Nmax, OP_T, t2, rk, Nb, rk, Nb));
    d2.push_back(gemm(R + (size_t)rk * Nmax, Nmax, OP_R, t2, rk, OP_N, core.as<double2>() + (size_t)b * rk * rk, rk,
                      rk, rk, Nb, -1.0));
  }
  CBFM_HIP(hipGetLastError());
  zgemm_batched(d1, s);
  zgemm_batched(d2, s);
  // SVD of the cores: right singular vectors U~ and U~ S^{-1}
  Scratch sv((size_t)nb * rk * sizeof(double), s);
  Scratch Ut((size_t)nb * rk * rk * sizeof(double2), s);
  Scratch Uts((size_t)nb * rk * rk * sizeof(double2), s);
  {
    const int ncmax = std::min(Nmax, rk);
    const size_t lds = (size_t)ncmax * ncmax * sizeof(double2) + (size_t)ncmax * (sizeof(double2) + 12);
    const double tol = std::sqrt((double)ncmax) * 2.220446049250313e-16;
    const int max_sweeps = 60;
    if (lds <= core_svd_lds_limit()) {
      hipLaunchKernelGGL(core_svd_kernel<true>, dim3(nb), dim3(1024), lds, s, core.as<double2>(), rk,
                         dN_p, nullptr, tol, max_sweeps, sv.as<double>(), Ut.as<double2>(),
                         Uts.as<double2>(), info.as<int32_t>());
    } else {
      Scratch work((size_t)nb * rk * rk * sizeof(double2), s);
      hipLaunchKernelGGL(core_svd_kernel<false>, dim3(nb), dim3(1024), (size_t)ncmax * (sizeof(double2) + 12), s,
                         core.as<double2>(), rk, dN_p, work.as<double2>(), tol, max_sweeps,
                         sv.as<double>(), Ut.as<double2>(), Uts.as<double2>(), info.as<int32_t>());
    }
    CBFM_HIP(hipGetLastError());
  }
  std::vector<double> hs((size_t)nb * rk);
  CBFM_HIP(hipMemcpyAsync(hs.data(), sv.p, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CBFM_HIP(hipMemcpyAsync(hinfo.data(), info.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CBFM_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < nb; ++b)
    CBFM_REQUIRE(hinfo[b] == 0, CBFM_E_HIP, "cell " + std::to_string(b) + ": Jacobi SVD did not converge");
  auto* c = new cbfm_cbf_s();
  try {
    c->mesh = m;
    c->L.resize(nb);
    for (int b = 0; b < nb; ++b) {
      const double* sb = &hs[(size_t)b * rk];
      int L = 0;
      const int Nb = hN[b];
      while (L < rk && L < Nb && sb[L] > 0 && sb[L] >= delta_svd * sb[0]) ++L;
      if (max_L > 0) L = std::min(L, max_L);
      CBFM_REQUIRE(L > 0, CBFM_E_RANK, "cell " + std::to_string(b) + " keeps no CBF");
      c->L[b] = L;
      c->sigma.insert(c->sigma.end(), sb, sb + L);
    }
    // translated copies of one cell: the plane waves on cell b are those on
    // cell 0 times one phase per wave, so its currents are cell 0's times
    // a diagonal phase matrix and its CBFs span cell 0's spaces; every
    // cell takes cell 0's (count, singular values and vectors)
    if (share) {
      c->shared = true;
      c->sigma.resize((size_t)c->L[0] * nb);
      for (int b = 1; b < nb; ++b) {
        c->L[b] = c->L[0];
        std::copy(c->sigma.begin(), c->sigma.begin() + c->L[0], c->sigma.begin() + (size_t)b * c->L[0]);
      }
    }
    cbf_finish(c);
    c->CM.alloc(std::max<int64_t>(1, c->coff[nb]) * sizeof(double2));
    c->CJ.alloc(std::max<int64_t>(1, c->coff[nb]) * sizeof(double2));
    // C^J = R_J^H V_L with V = U~;  C^M = R_M^H U_L with U = X V S^{-1} = X U~ S^{-1}
    Scratch W((size_t)std::max<int64_t>(1, c->coff[nb]) * sizeof(double2), s);
    std::vector<GemmDesc> d3, d4;
    for (int b = 0; b < nb; ++b) {
      const int Nb = hN[b], nc = std::min(Nb, rk), L = c->L[b];
      const double2* R = Rf.as<double2>() + (size_t)b * 2 * rk * Nmax;
      const double2* ub = Ut.as<double2>() + (size_t)b * rk * rk;
      const double2* usb = Uts.as<double2>() + (size_t)b * rk * rk;
      double2* wb = W.as<double2>() + c->coff[b];  // nc x L row-major (nc <= N_b)
      d3.push_back(gemm(core.as<double2>() + (size_t)b * rk * rk, rk, OP_T, usb, rk, OP_T, wb, L, nc, L, nc));
      d3.push_back(gemm(R + (size_t)rk * Nmax, Nmax, OP_C, ub, rk, OP_T, c->CJ.as<double2>() + c->coff[b], L, Nb, L,
                        nc));
      d4.push_back(gemm(R, Nmax, OP_C, wb, L, OP_N, c->CM.as<double2>() + c->coff[b], L, Nb, L, nc));
    }
    zgemm_batched(d3, s);
    zgemm_batched(d4, s);
    if (c->shared) {
      const size_t blk = (size_t)(c->coff[1] - c->coff[0]) * sizeof(double2);
      for (int b = 1; b < nb; ++b) {
        CBFM_HIP(hipMemcpyAsync(c->CM.as<double2>() + c->coff[b], c->CM.as<double2>(), blk,
                                hipMemcpyDeviceToDevice, s));
        CBFM_HIP(hipMemcpyAsync(c->CJ.as<double2>() + c->coff[b], c->CJ.as<double2>(), blk,
                                hipMemcpyDeviceToDevice, s));
      }
    }
    if (t_async_cmp) cmp_factor_async(c, s);
  } catch (...) {
    delete c;
    throw;
  }
  return c;
}

// From whole-body current coefficients (IPCBF): vector c of X (length 2 ne,
// the library's cell order) holds [alpha^M; alpha^J] of wave c; cell b's
// rows give (J^M_b)^H and (J^J_b)^H, column-major S x Nmax (QA layout).
__global__ void pack_global_kernel(const double2* __restrict__ X, int64_t ne, int S, const int64_t* __restrict__ cell_off,
                                   int Nmax, double2* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y, b = blockIdx.z >> 1, w = blockIdx.z & 1;
  if (r >= S) return;
  const int64_t c0 = cell_off[b], N = cell_off[b + 1] - c0;
  double2 x = make_double2(0.0, 0.0);
  if (i < N) {
    x = X[(int64_t)r * 2 * ne + (int64_t)w * ne + c0 + i];
    x.y = -x.y;
  }
  out[((int64_t)(2 * b + w) * Nmax + i) * S + r] = x;
}

cbfm_cbf_s* cbfm::cbf_from_currents(const cbfm_mesh_s* m, const double2* X, int S, double delta_svd, int max_L,
                                    hipStream_t s) {
  const MeshHost& h = m->h;
  const int nb = h.nblocks;
  int Nmax = 0;
  std::vector<int32_t> hN(nb);
  for (int b = 0; b < nb; ++b) {
    hN[b] = (int32_t)(h.cell_off[b + 1] - h.cell_off[b]);
    Nmax = std::max<int>(Nmax, hN[b]);
  }
  // per cell its RWGs (the segment of the cell-order table) for the Gram
  std::vector<CellJob> jobs(nb);
  for (int b = 0; b < nb; ++b) {
    jobs[b] = CellJob{};
    jobs[b].N = hN[b];
    jobs[b].edges = m->perm.as<int32_t>() + h.cell_off[b];
  }
  Scratch dN((size_t)nb * sizeof(int32_t), s), djobs((size_t)nb * sizeof(CellJob), s),
      dco((size_t)(nb + 1) * sizeof(int64_t), s);
  CBFM_HIP(hipMemcpyAsync(dN.p, hN.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, s));
  CBFM_HIP(hipMemcpyAsync(djobs.p, jobs.data(), nb * sizeof(CellJob), hipMemcpyHostToDevice, s));
  CBFM_HIP(hipMemcpyAsync(dco.p, h.cell_off.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  Scratch QA((size_t)nb * 2 * S * Nmax * sizeof(double2), s);
  hipLaunchKernelGGL(pack_global_kernel, dim3((S + 255) / 256, Nmax, 2 * nb), dim3(256), 0, s, X, h.ne, S,
                     dco.as<int64_t>(), Nmax, QA.as<double2>());
  CBFM_HIP(hipGetLastError());
  cbfm_cbf_s* c = orthogonalise(m, QA.as<double2>(), S, Nmax, hN, dN.as<int32_t>(), djobs.as<CellJob>(), delta_svd,
                                max_L, false, s);
  CBFM_HIP(hipStreamSynchronize(s));  // host tables of this frame
  return c;
}

extern "C" {

cbfm_status cbfm_build_cbf(cbfm_mesh m, const cbfm_medium* med, const cbfm_cbf_params* prm, void* stream,
                           cbfm_cbf* out) {
  return guarded([&] {
    CBFM_REQUIRE(m && prm && out, CBFM_E_ARG, "null argument");
    *out = nullptr;
    CBFM_REQUIRE(prm->gen_host && prm->n_gen > 0, CBFM_E_ARG, "need generating waves");
    CBFM_REQUIRE(prm->delta_svd >= 0 && prm->delta_svd <= 1, CBFM_E_ARG, "delta_svd outside [0, 1]");
    CBFM_REQUIRE(prm->n_gen <= 4096, CBFM_E_ARG, "n_gen above 4096");
    const Media md = make_media(med);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MeshHost& h = m->h;
    const int nb = h.nblocks;
    const int S = prm->n_gen;
    int Nmax = 0;
    for (int b = 0; b < nb; ++b) Nmax = std::max<int>(Nmax, (int)(h.cell_off[b + 1] - h.cell_off[b]));
    const int n = 2 * Nmax;
    CBFM_REQUIRE(nb <= 32767 && n <= 65535, CBFM_E_ARG, "above 32767 cells or 32767 RWGs in one cell");
    // generating right-hand sides on all edges
    Scratch vgen((size_t)S * 2 * h.ne * sizeof(double2), s);
    Scratch dinc((size_t)S * 6 * sizeof(double), s);
    CBFM_HIP(hipMemcpyAsync(dinc.p, prm->gen_host, (size_t)S * 6 * sizeof(double), hipMemcpyHostToDevice, s));
    rhs_launch(m, md, med->eta0, dinc.as<double>(), S, vgen.p, s);
    // per cell the augmented system [Z_mm | V_m] (padded, row-major n x (n + S))
    const int ldz = n + S;
    Scratch Aug((size_t)nb * n * ldz * sizeof(double2), s);
    std::vector<CellSupport> cs = supports(h, nb);
    // groups of cells whose triangle-local blocks fit in at most 1 GiB (or
    // one cell), filled together; each cell's blocks at loff[b] elements
    size_t maxloc = 0;
    for (int b = 0; b < nb; ++b) maxloc = std::max(maxloc, cs[b].tris.size());
    const size_t group_bytes = std::max<size_t>((size_t)1 << 30, (size_t)27 * maxloc * maxloc * sizeof(double2));
    std::vector<int> gstart{0};
    std::vector<size_t> gbytes;
    std::vector<int64_t> loff(nb);
    {
      size_t bytes = 0;
      for (int b = 0; b < nb; ++b) {
        const size_t cb = (size_t)27 * cs[b].tris.size() * cs[b].tris.size() * sizeof(double2);
        if (b > gstart.back() && bytes + cb > group_bytes) {
          gbytes.push_back(bytes);
          gstart.push_back(b);
          bytes = 0;
        }
        loff[b] = (int64_t)(bytes / sizeof(double2));
        bytes += cb;
      }
      gbytes.push_back(bytes);
      gstart.push_back(nb);
    }
    // index staging for every cell, uploaded once: support lists, the near
    // pairs of all cells in one array (each tagged with its cell), and the
    // per-cell tables of the batched launches
    std::vector<int64_t> noff(nb + 1, 0);
    for (int b = 0; b < nb; ++b) noff[b + 1] = noff[b] + (int64_t)cs[b].near.size();
    auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
    size_t ibytes = al(sizeof(NearPair) * noff[nb]) + al(sizeof(CellJob) * nb) + al(sizeof(NearOut) * nb);
    for (int b = 0; b < nb; ++b) ibytes += al(4 * cs[b].tris.size()) + al(4 * cs[b].pos.size()) + al(4 * cs[b].edges.size());
    std::vector<char> host(ibytes);
    Scratch idx(ibytes, s);
    size_t o = 0;
    auto put = [&](const void* src, size_t bytes) {
      if (bytes) std::memcpy(host.data() + o, src, bytes);
      void* d = idx.as<char>() + o;
      o += al(bytes);
      return d;
    };
    std::vector<const int32_t*> dtris(nb);
    std::vector<CellJob> jobs(nb);
    std::vector<NearOut> nouts(nb);
    for (int b = 0; b < nb; ++b) {
      const int64_t nt_b = (int64_t)cs[b].tris.size();
      dtris[b] = (const int32_t*)put(cs[b].tris.data(), 4 * cs[b].tris.size());
      jobs[b].pos = (const int32_t*)put(cs[b].pos.data(), 4 * cs[b].pos.size());
      jobs[b].edges = (const int32_t*)put(cs[b].edges.data(), 4 * cs[b].edges.size());
      jobs[b].loff = loff[b];
      jobs[b].nt = (int32_t)nt_b;
      jobs[b].N = (int32_t)cs[b].edges.size();
      nouts[b] = {loff[b], 9 * nt_b * nt_b, 3 * nt_b};
      for (NearPair& q : cs[b].near) q.pad = b;
    }
    NearPair* dnear = (NearPair*)(idx.as<char>() + o);
    for (int b = 0; b < nb; ++b) {
      std::memcpy(host.data() + o, cs[b].near.data(), sizeof(NearPair) * cs[b].near.size());
      o += sizeof(NearPair) * cs[b].near.size();
    }
    o = al(o);
    const CellJob* djobs = (const CellJob*)put(jobs.data(), sizeof(CellJob) * nb);
    const NearOut* douts = (const NearOut*)put(nouts.data(), sizeof(NearOut) * nb);
    CBFM_REQUIRE(o == ibytes, CBFM_E_HIP, "cell index staging size mismatch");
    CBFM_HIP(hipMemcpyAsync(idx.p, host.data(), ibytes, hipMemcpyHostToDevice, s));
    // the cells' self blocks, a group at a time: regular pairs in one
    // persistent launch, the near pairs of all the group's cells in one
    // launch pair, then assembly and packing of every cell in one launch
    for (size_t g = 0; g + 1 < gstart.size(); ++g) {
      const int g0 = gstart[g], g1 = gstart[g + 1];
      Scratch local(gbytes[g], s);
      std::vector<FillBatchItem> items;
      for (int b = g0; b < g1; ++b) {
        const int64_t nt_b = cs[b].tris.size();
        items.push_back({m, md, CBFM_LAYOUT_OPS3, dtris[b], nt_b, dtris[b], nt_b, local.as<double2>() + loff[b]});
      }
      fill_regular_batch(items, CBFM_FP64, s);
      fill_near_batch(m, md, CBFM_LAYOUT_OPS3, dnear + noff[g0], noff[g1] - noff[g0], douts + g0, g0, local.p, s);
      hipLaunchKernelGGL(cell_zmm_kernel, dim3((n + 255) / 256, n, g1 - g0), dim3(256), 0, s, local.as<double2>(),
                         djobs, g0, m->tplus.as<int32_t>(), m->tminus.as<int32_t>(), m->aplus.as<int32_t>(),
                         m->aminus.as<int32_t>(), n, ldz, Aug.as<double2>());
      CBFM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(cell_v_kernel, dim3((S + 255) / 256, n, nb), dim3(256), 0, s, vgen.as<double2>(), h.ne, djobs,
                       n, S, Aug.as<double2>());
    CBFM_HIP(hipGetLastError());
    // Z_mm J_m = V_m for every cell (Gauss-Jordan on the augmented systems)
    gj_solve_batched(Aug.as<double2>(), (int64_t)n * ldz, ldz, n, ldz, nb, "Z_mm of cell", s);
    // QR of (J^M)^H and (J^J)^H (column-major S x Nmax, zero-padded)
    std::vector<int32_t> hN(nb);
    for (int b = 0; b < nb; ++b) hN[b] = (int32_t)cs[b].edges.size();
    Scratch dN((size_t)nb * sizeof(int32_t), s);
    CBFM_HIP(hipMemcpyAsync(dN.p, hN.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, s));
    Scratch QA((size_t)nb * 2 * S * Nmax * sizeof(double2), s);
    hipLaunchKernelGGL(pack_jh_kernel, dim3((S + 255) / 256, Nmax, 2 * nb), dim3(256), 0, s, Aug.as<double2>(), n,
                       S, dN.as<int32_t>(), Nmax, QA.as<double2>());
    CBFM_HIP(hipGetLastError());
    cbfm_cbf_s* c = orthogonalise(m, QA.as<double2>(), S, Nmax, hN, dN.as<int32_t>(), djobs, prm->delta_svd,
                                  prm->max_L, m->translated, s);
    *out = c;
  });
}

cbfm_status cbfm_cbf_import(cbfm_mesh m, const int32_t* L, const void* CM, const void* CJ, const double* sigma,
                            void* stream, cbfm_cbf* out) {
  return guarded([&] {
    CBFM_REQUIRE(m && L && CM && CJ && sigma && out, CBFM_E_ARG, "null argument");
    *out = nullptr;
    const MeshHost& h = m->h;
    auto* c = new cbfm_cbf_s();
    try {
      c->mesh = m;
      c->L.assign(L, L + h.nblocks);
      for (int b = 0; b < h.nblocks; ++b) {
        const int64_t Nb = h.cell_off[b + 1] - h.cell_off[b];
        CBFM_REQUIRE(c->L[b] > 0 && c->L[b] <= Nb, CBFM_E_ARG, "L out of range for cell " + std::to_string(b));
      }
      cbf_finish(c);
      c->sigma.assign(sigma, sigma + c->NL);
      const size_t bytes = c->coff[h.nblocks] * sizeof(double2);
      c->CM.alloc(bytes);
      c->CJ.alloc(bytes);
      CBFM_HIP(hipMemcpy(c->CM.p, CM, bytes, hipMemcpyHostToDevice));
      CBFM_HIP(hipMemcpy(c->CJ.p, CJ, bytes, hipMemcpyHostToDevice));
      (void)stream;
      // on a mesh of translated copies of cell 0, CBFs equal to cell 0's in
      // every cell are shared (the projection then goes by cell offsets)
      if (m->translated) {
        const int nb = h.nblocks;
        const size_t blk = (size_t)(c->coff[1] - c->coff[0]) * sizeof(double2);
        bool same = true;
        for (int b = 1; b < nb && same; ++b)
          same = c->L[b] == c->L[0] &&
                 std::memcmp((const char*)CM + c->coff[b] * sizeof(double2), CM, blk) == 0 &&
                 std::memcmp((const char*)CJ + c->coff[b] * sizeof(double2), CJ, blk) == 0;
        c->shared = same;
      }
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

cbfm_status cbfm_cbf_info(cbfm_cbf c, int64_t* n_cbf, int32_t* L, double* sigma) {
  return guarded([&] {
    CBFM_REQUIRE(c != nullptr, CBFM_E_ARG, "cbf is NULL");
    if (n_cbf) *n_cbf = 2 * c->NL;
    if (L) std::memcpy(L, c->L.data(), c->L.size() * sizeof(int32_t));
    if (sigma) std::memcpy(sigma, c->sigma.data(), c->sigma.size() * sizeof(double));
  });
}

cbfm_status cbfm_cbf_export(cbfm_cbf c, void* CM, void* CJ) {
  return guarded([&] {
    CBFM_REQUIRE(c != nullptr, CBFM_E_ARG, "cbf is NULL");
    const size_t bytes = c->coff.back() * sizeof(double2);
    if (CM) CBFM_HIP(hipMemcpy(CM, c->CM.p, bytes, hipMemcpyDeviceToHost));
    if (CJ) CBFM_HIP(hipMemcpy(CJ, c->CJ.p, bytes, hipMemcpyDeviceToHost));
  });
}

void cbfm_cbf_free(cbfm_cbf c) { delete c; }

cbfm_status cbfm_cmp_apply(cbfm_cbf c, int64_t nrhs, const void* y, void* x, void* stream) {
  return cbfm_cmp_apply_ex(c, nrhs, y, x, CBFM_CMP_EXACT, 0.0, stream);
}

cbfm_status cbfm_cmp_apply_ex(cbfm_cbf c, int64_t nrhs, const void* y, void* x, int32_t mode, double inner_tol,
                              void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(c && y && x && nrhs >= 0, CBFM_E_ARG, "bad argument");
    CBFM_REQUIRE(mode == CBFM_CMP_EXACT || mode == CBFM_CMP_INNER_GMRES, CBFM_E_ARG, "unknown CMP mode");
    CBFM_REQUIRE(mode == CBFM_CMP_EXACT || (inner_tol >= 0 && inner_tol < 1), CBFM_E_ARG, "inner_tol outside [0, 1)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)nrhs * 2 * c->NL * sizeof(double2);
    if (mode == CBFM_CMP_INNER_GMRES) {
      Scratch yc(bytes, s);  // (x and y may alias)
      CBFM_HIP(hipMemcpyAsync(yc.p, y, bytes, hipMemcpyDeviceToDevice, s));
      cmp_inner_apply(c, nrhs, yc.as<double2>(), static_cast<double2*>(x), inner_tol > 0 ? inner_tol : 1e-5, s);
      return;
    }
    if (x != y) CBFM_HIP(hipMemcpyAsync(x, y, bytes, hipMemcpyDeviceToDevice, s));
    cmp_apply_dev(c, nrhs, static_cast<double2*>(x), s);
  });
}

}  // extern "C"
