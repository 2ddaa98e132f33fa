// Reduced solve and RCS (paper Sec. III-C outer/inner CBFM equations and
// the current reconstruction; monostatic RCS after Knott).
//
//   v_r = (C^JM)^H v                   (tested incident fields, projected)
//   GMRES on  Z_r (G^CBF)^{-1} y = v_r, x0 = 0, restarted   (right precond.)
//   j_CBF = (G^CBF)^{-1} y,   j = C^MJ j_CBF
//   sigma = k0^2 / (4 pi) |eta0 N_perp - rhat x L|^2
//
// GMRES runs on the device for all right-hand sides at once, each with its
// own Krylov space (Saad's GMRES; classical Gram-Schmidt with selective
// re-orthogonalisation; complex Givens rotations).  Matrix-vector products are matrix-core
// GEMMs over all right-hand sides; the Hessenberg updates run one thread per
// right-hand side.  The host only reads the convergence flags each step.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cbf.h"
#include "gemm.h"

namespace cbfm {

// ------------------------------------------------------------- small kernels
// out[c][i] = in[c][perm[i]] (gather, forward) or out[c][perm[i]] = in[c][i]
// for both halves of 2ne-long vectors
__global__ void permute_kernel(const double2* __restrict__ in, double2* __restrict__ out, const int32_t* __restrict__ perm,
                               int64_t ne, int64_t nv, int forward) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (i >= ne || c >= nv) return;
  const int64_t base = c * 2 * ne;
  const int64_t p = perm[i];
  if (forward) {
    out[base + i] = in[base + p];
    out[base + ne + i] = in[base + ne + p];
  } else {
    out[base + p] = in[base + i];
    out[base + ne + p] = in[base + ne + i];
  }
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Sum over a block of 256 threads, the same order on every call.
__device__ inline double block_sum256(double s, double* sh) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __syncthreads();  // sh may still be read from a previous call
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// h[i * nrhs + c] = sum_k conj(V[i][c][k]) u[c][k] for i < jp1 and, with
// self != 0, h[jp1 * nrhs + c] = ||u[c]||^2; one wavefront per dot product,
// four per block, only for right-hand sides with flag[c].
__global__ void __launch_bounds__(256) dots_kernel(const double2* __restrict__ V, int64_t vstride,
                                                   const double2* __restrict__ u, int64_t n, int64_t nrhs, int64_t jp1,
                                                   int self, const int32_t* __restrict__ flag,
                                                   double2* __restrict__ h) {
  const int64_t id = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (id >= (jp1 + self) * nrhs) return;
  const int64_t i = id / nrhs, c = id % nrhs;
  if (!flag[c]) return;
  const double2* v = i < jp1 ? V + i * vstride + c * n : u + c * n;
  const double2* w = u + c * n;
  double re = 0, im = 0;
  for (int64_t k = lane; k < n; k += 64) {
    const double2 a = v[k], b = w[k];
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) h[i * nrhs + c] = make_double2(re, im);
}

// One classical Gram-Schmidt update u[c] -= sum_{i<jp1} h[i][c] V[i][c] for
// the right-hand sides with flag[c]; each block stores the partial sum of
// |u|^2 over its rows in part[c * gridDim.x + blockIdx.x].  Block 0 of each
// right-hand side also
//  - first pass (mask given): sets mask[c] when the projection removed more
//    than half of the squared norm, sum_i |h_i|^2 > ||u||^2 / 2 with ||u||^2
//    in h[jp1] -- the Daniel-Gragg-Kaufman-Stewart test (after < before /
//    sqrt 2) for a second pass;
//  - second pass (hsum given): adds h into hsum, so that the Hessenberg column
//    is the sum of both passes.
__global__ void __launch_bounds__(256) orth_update_kernel(const double2* __restrict__ V, int64_t vstride,
                                                          double2* __restrict__ u, int64_t n, int64_t jp1, int64_t nrhs,
                                                          const int32_t* __restrict__ flag, const double2* h,
                                                          double* __restrict__ part, int32_t* __restrict__ mask,
                                                          double2* hsum) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (!flag[c]) {  // uniform over the block
    if (mask && blockIdx.x == 0 && threadIdx.x == 0) mask[c] = 0;
    return;
  }
  __shared__ double sh[4];
  double s = 0;
  if (k < n) {
    double2 acc = u[c * n + k];
#pragma unroll 4
    for (int64_t i = 0; i < jp1; ++i) {
      const double2 a = h[i * nrhs + c], v = V[i * vstride + c * n + k];
      acc.x -= a.x * v.x - a.y * v.y;
      acc.y -= a.x * v.y + a.y * v.x;
    }
    u[c * n + k] = acc;
    s = acc.x * acc.x + acc.y * acc.y;
  }
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) part[c * gridDim.x + blockIdx.x] = s;
  if (blockIdx.x != 0) return;
  if (mask) {
    double q = 0;
    for (int64_t i = threadIdx.x; i < jp1; i += blockDim.x) {
      const double2 a = h[i * nrhs + c];
      q += a.x * a.x + a.y * a.y;
    }
    q = block_sum256(q, sh);
    if (threadIdx.x == 0) mask[c] = q > 0.5 * h[jp1 * nrhs + c].x ? 1 : 0;
  }
  if (hsum)
    for (int64_t i = threadIdx.x; i < jp1; i += blockDim.x) hsum[i * nrhs + c] = cadd(hsum[i * nrhs + c], h[i * nrhs + c]);
}

// nrm[c] = sqrt(sum of the np partial sums of |u[c]|^2); out[c] = u[c] / nrm[c]
// (zero if nrm[c] == 0); only right-hand sides with flag[c]
__global__ void normalize_kernel(const double2* __restrict__ u, double2* __restrict__ out, int64_t n,
                                 const double* __restrict__ part, int np, double* __restrict__ nrm,
                                 const int32_t* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (!flag[c]) return;
  double q = 0;
  for (int b = 0; b < np; ++b) q += part[c * np + b];
  const double nr = sqrt(q);
  if (blockIdx.x == 0 && threadIdx.x == 0) nrm[c] = nr;
  if (k >= n) return;
  const double sc = nr > 0 ? 1.0 / nr : 0.0;
  const double2 a = u[c * n + k];
  out[c * n + k] = make_double2(a.x * sc, a.y * sc);
}

// nrm[c] = ||u[c]|| (one block per vector); skipped for inactive vectors
__global__ void __launch_bounds__(256) norm_kernel(const double2* __restrict__ u, int64_t n, double* __restrict__ nrm,
                                                   const int32_t* __restrict__ active) {
  const int64_t c = blockIdx.x;
  if (active && !active[c]) return;
  double s = 0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const double2 a = u[c * n + k];
    s += a.x * a.x + a.y * a.y;
  }
  __shared__ double sh[4];
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) nrm[c] = sqrt(s);
}

// out[c] = in[c] / nrm[c] (zero if nrm[c] == 0)
__global__ void scale_kernel(const double2* __restrict__ in, double2* __restrict__ out, int64_t n,
                             const double* __restrict__ nrm) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (k >= n) return;
  const double s = nrm[c] > 0 ? 1.0 / nrm[c] : 0.0;
  const double2 a = in[c * n + k];
  out[c * n + k] = make_double2(a.x * s, a.y * s);
}

// r = b - r
__global__ void sub_from_kernel(const double2* __restrict__ b, double2* __restrict__ r, int64_t total) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  r[k] = make_double2(b[k].x - r[k].x, b[k].y - r[k].y);
}

// Per right-hand side state, right-hand side index fastest (coalesced).
struct GmresState {
  double2* H;      // column j, row i at [(j * (m + 1) + i) * nrhs + c]
  double2* cs;     // [i * nrhs + c]
  double2* sn;     // [i * nrhs + c]
  double2* g;      // [i * nrhs + c], i <= m
  double2* hcol;   // new column, [i * nrhs + c]
  double* nrm;     // [c]
  double* bnorm;   // [c]
  double* res;     // [c] residual estimate / bnorm
  int32_t* active; // [c]
  int32_t* kc;     // [c] Krylov dimension reached in this cycle
  int32_t* its;    // [c] iterations spent (all cycles)
};

// Start a cycle: g = beta e1, active = beta/bnorm > tol, kc = 0.
__global__ void cycle_init_kernel(GmresState st, int64_t m, int64_t nrhs, double tol) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double beta = st.nrm[c];
  for (int64_t i = 0; i <= m; ++i) st.g[i * nrhs + c] = make_double2(0, 0);
  st.g[c] = make_double2(beta, 0);
  const double r = st.bnorm[c] > 0 ? beta / st.bnorm[c] : 0.0;
  st.res[c] = r;
  st.active[c] = r > tol ? 1 : 0;
  st.kc[c] = 0;
}

// Column j of the Hessenberg matrix from hcol (rows 0..j) and nrm (row j+1):
// apply the previous rotations, form the new one, update g, test convergence.
// One wavefront per right-hand side.  Rotation i maps (a_i, h_{i+1}) to
// (c_i a_i + s_i h_{i+1}, a_{i+1}) with a_{i+1} = -conj(s_i) a_i + conj(c_i)
// h_{i+1}, a_0 = h_0: the carried a_i follow an affine recurrence, so each
// lane composes the maps of a contiguous run of rotations, a scan over the
// lanes gives every run its incoming a_i, and the runs are then replayed in
// parallel.
__global__ void __launch_bounds__(256) givens_kernel(GmresState st, int64_t m, int64_t j, int64_t nrhs, double tol) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nrhs || !st.active[c]) return;  // uniform over the wavefront
  const int64_t K = (j + 63) / 64;
  const int64_t i0 = std::min<int64_t>(j, lane * K), i1 = std::min<int64_t>(j, i0 + K);
  double2 P = make_double2(1, 0), Q = make_double2(0, 0);
  for (int64_t i = i0; i < i1; ++i) {
    const double2 sn = st.sn[i * nrhs + c], cs = st.cs[i * nrhs + c], b = st.hcol[(i + 1) * nrhs + c];
    const double2 Pi = make_double2(-sn.x, sn.y);  // -conj(s_i)
    const double2 Qi = cmul(make_double2(cs.x, -cs.y), b);
    Q = cadd(cmul(Pi, Q), Qi);
    P = cmul(Pi, P);
  }
  // inclusive scan: after it, (P, Q) maps a_0 to the carry leaving this run
  for (int off = 1; off < 64; off <<= 1) {
    const double2 Po = make_double2(__shfl_up(P.x, off, 64), __shfl_up(P.y, off, 64));
    const double2 Qo = make_double2(__shfl_up(Q.x, off, 64), __shfl_up(Q.y, off, 64));
    if (lane >= off) {
      Q = cadd(cmul(P, Qo), Q);
      P = cmul(P, Po);
    }
  }
  const double2 a0 = st.hcol[c];
  const double2 Pe = make_double2(__shfl_up(P.x, 1, 64), __shfl_up(P.y, 1, 64));
  const double2 Qe = make_double2(__shfl_up(Q.x, 1, 64), __shfl_up(Q.y, 1, 64));
  double2 a = lane == 0 ? a0 : cadd(cmul(Pe, a0), Qe);
  for (int64_t i = i0; i < i1; ++i) {
    const double2 sn = st.sn[i * nrhs + c], cs = st.cs[i * nrhs + c], b = st.hcol[(i + 1) * nrhs + c];
    st.H[(j * (m + 1) + i) * nrhs + c] = cadd(cmul(cs, a), cmul(sn, b));
    a = cadd(cmul(make_double2(-sn.x, sn.y), a), cmul(make_double2(cs.x, -cs.y), b));
  }
  const int last = j == 0 ? 0 : (int)((j - 1) / K);  // lane that ends with a_j
  a = make_double2(__shfl(a.x, last, 64), __shfl(a.y, last, 64));
  if (lane != 0) return;
  const double2 b = make_double2(st.nrm[c], 0);
  const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x);
  double2 cc = make_double2(1, 0), ss = make_double2(0, 0);
  if (den > 0) {
    cc = make_double2(a.x / den, -a.y / den);  // conj(a)/den
    ss = make_double2(b.x / den, 0.0);         // conj(b)/den, b real
  }
  st.cs[j * nrhs + c] = cc;
  st.sn[j * nrhs + c] = ss;
  st.H[(j * (m + 1) + j) * nrhs + c] = make_double2(den, 0);
  const double2 gj = st.g[j * nrhs + c];
  // g[j+1] = -conj(s) g[j];  g[j] = c g[j]
  const double2 gn = make_double2(-(ss.x * gj.x + ss.y * gj.y), -(ss.x * gj.y - ss.y * gj.x));
  st.g[(j + 1) * nrhs + c] = gn;
  st.g[j * nrhs + c] = make_double2(cc.x * gj.x - cc.y * gj.y, cc.x * gj.y + cc.y * gj.x);
  const double r = sqrt(gn.x * gn.x + gn.y * gn.y) / st.bnorm[c];
  st.res[c] = r;
  st.kc[c] = (int32_t)(j + 1);
  st.its[c] += 1;
  if (r <= tol || den == 0.0) st.active[c] = 0;
}

// y = H^{-1} g over the first kc[c] rows (upper triangular), in place in g;
// one block per right-hand side, column-oriented back substitution.
__global__ void __launch_bounds__(256) backsolve_kernel(GmresState st, int64_t m, int64_t nrhs) {
  const int64_t c = blockIdx.x;
  const int64_t k = st.kc[c];
  __shared__ double2 yi;
  for (int64_t i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double2 s = st.g[i * nrhs + c], d = st.H[(i * (m + 1) + i) * nrhs + c];
      const double dd = d.x * d.x + d.y * d.y;
      yi = dd > 0 ? make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd) : make_double2(0, 0);
      st.g[i * nrhs + c] = yi;
    }
    __syncthreads();
    const double2 y = yi;
    for (int64_t t = threadIdx.x; t < i; t += blockDim.x) {
      const double2 h = st.H[(i * (m + 1) + t) * nrhs + c];
      double2* gt = st.g + t * nrhs + c;
      gt->x -= h.x * y.x - h.y * y.y;
      gt->y -= h.x * y.y + h.y * y.x;
    }
    __syncthreads();
  }
}

// x[c] += sum_{i < kc[c]} y[i][c] V[i][c]
__global__ void x_update_kernel(GmresState st, const double2* __restrict__ V, int64_t vstride, double2* __restrict__ x,
                                int64_t n, int64_t nrhs) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (k >= n) return;
  const int64_t kc = st.kc[c];
  double2 acc = x[c * n + k];
  for (int64_t i = 0; i < kc; ++i) {
    const double2 a = st.g[i * nrhs + c], v = V[i * vstride + c * n + k];
    acc.x += a.x * v.x - a.y * v.y;
    acc.y += a.x * v.y + a.y * v.x;
  }
  x[c * n + k] = acc;
}

// ------------------------------------------------------------- far field
// One block per (rhs, direction): radiation vectors N (from alpha^J) and L
// (from alpha^M) over all triangles and quadrature points, then sigma.
struct FarArgs {
  const double* xyz9;
  const int32_t* tri_edge;
  const double* c64;   // s_a l_a, [a * nt + t]
  int64_t nt, ne;
  double bary[7][3];
  double w[7];
  double k0, eta0;
};

__global__ void __launch_bounds__(256) farfield_kernel(FarArgs fa, const double2* __restrict__ j, const double* __restrict__ dirs,
                                                       const double* __restrict__ pol, int64_t ndir,
                                                       double* __restrict__ sigma) {
  const int64_t d = blockIdx.x, c = blockIdx.y;
  const double r[3] = {dirs[(c * ndir + d) * 3], dirs[(c * ndir + d) * 3 + 1], dirs[(c * ndir + d) * 3 + 2]};
  const double2* aM = j + c * 2 * fa.ne;
  const double2* aJ = aM + fa.ne;
  double acc[12] = {0};  // N (re, im) x3, L (re, im) x3
  for (int64_t t = threadIdx.x; t < fa.nt; t += blockDim.x) {
    const double* P = fa.xyz9 + t * 9;
    double2 cJ[3], cM[3];
    for (int a = 0; a < 3; ++a) {
      const int e = fa.tri_edge[t * 3 + a];
      const double ca = fa.c64[a * fa.nt + t] * 0.5;  // int_T f = sum_k w_k A (c/2A)(r - p) -> c/2
      cJ[a] = make_double2(aJ[e].x * ca, aJ[e].y * ca);
      cM[a] = make_double2(aM[e].x * ca, aM[e].y * ca);
    }
    for (int k = 0; k < 7; ++k) {
      double rk[3];
      for (int x = 0; x < 3; ++x) rk[x] = fa.bary[k][0] * P[x] + fa.bary[k][1] * P[3 + x] + fa.bary[k][2] * P[6 + x];
      double sn, cs;
      sincos(fa.k0 * (r[0] * rk[0] + r[1] * rk[1] + r[2] * rk[2]), &sn, &cs);  // e^{+j k0 r.r'}
      const double wk = fa.w[k];
      for (int a = 0; a < 3; ++a) {
        const double2 pJ = make_double2(wk * (cJ[a].x * cs - cJ[a].y * sn), wk * (cJ[a].x * sn + cJ[a].y * cs));
        const double2 pM = make_double2(wk * (cM[a].x * cs - cM[a].y * sn), wk * (cM[a].x * sn + cM[a].y * cs));
        for (int x = 0; x < 3; ++x) {
          const double dv = rk[x] - P[a * 3 + x];
          acc[2 * x] += pJ.x * dv;
          acc[2 * x + 1] += pJ.y * dv;
          acc[6 + 2 * x] += pM.x * dv;
          acc[6 + 2 * x + 1] += pM.y * dv;
        }
      }
    }
  }
  __shared__ double sh[12][256];
  for (int q = 0; q < 12; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 12; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double N[3][2], L[3][2];
    for (int x = 0; x < 3; ++x) {
      N[x][0] = sh[2 * x][0];
      N[x][1] = sh[2 * x + 1][0];
      L[x][0] = sh[6 + 2 * x][0];
      L[x][1] = sh[6 + 2 * x + 1][0];
    }
    const double rn[2] = {r[0] * N[0][0] + r[1] * N[1][0] + r[2] * N[2][0], r[0] * N[0][1] + r[1] * N[1][1] + r[2] * N[2][1]};
    double F[3][2];
    for (int x = 0; x < 3; ++x) {
      const int x1 = (x + 1) % 3, x2 = (x + 2) % 3;
      for (int p = 0; p < 2; ++p) {
        const double nperp = N[x][p] - r[x] * rn[p];
        const double rxl = r[x1] * L[x2][p] - r[x2] * L[x1][p];
        F[x][p] = fa.eta0 * nperp - rxl;
      }
    }
    double s2;
    if (pol) {
      const double* pp = pol + (c * ndir + d) * 3;
      const double fr = F[0][0] * pp[0] + F[1][0] * pp[1] + F[2][0] * pp[2];
      const double fi = F[0][1] * pp[0] + F[1][1] * pp[1] + F[2][1] * pp[2];
      s2 = fr * fr + fi * fi;
    } else {
      s2 = 0;
      for (int x = 0; x < 3; ++x) s2 += F[x][0] * F[x][0] + F[x][1] * F[x][1];
    }
    sigma[c * ndir + d] = fa.k0 * fa.k0 / (4.0 * M_PI) * s2;
  }
}

// Device flags read back through pinned host memory: post() queues a copy
// and an event, wait() blocks on the last posted copy; sync_read() copies and
// waits at once.
struct PinnedFlags {
  int64_t n;
  int32_t* host = nullptr;
  hipEvent_t ev = nullptr;
  bool posted = false;
  explicit PinnedFlags(int64_t count) : n(count) {
    CBFM_HIP(hipHostMalloc((void**)&host, n * sizeof(int32_t), hipHostMallocDefault));
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(host);
      throw Error{CBFM_E_HIP, "hipEventCreate failed"};
    }
  }
  ~PinnedFlags() {
    if (posted) (void)hipEventSynchronize(ev);
    (void)hipEventDestroy(ev);
    (void)hipHostFree(host);
  }
  PinnedFlags(const PinnedFlags&) = delete;
  PinnedFlags& operator=(const PinnedFlags&) = delete;
  void post(const int32_t* dev, hipStream_t s) {
    CBFM_HIP(hipMemcpyAsync(host, dev, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CBFM_HIP(hipEventRecord(ev, s));
    posted = true;
  }
  const int32_t* wait() {
    if (posted) CBFM_HIP(hipEventSynchronize(ev));
    posted = false;
    return host;
  }
  const int32_t* sync_read(const int32_t* dev, hipStream_t s) {
    post(dev, s);
    return wait();
  }
};

static dim3 grid2(int64_t n, int64_t m) { return dim3((unsigned)((n + 255) / 256), (unsigned)m); }

// u = A w for row-stored vectors w (nrhs x n): u^T = A w^T.
static void apply_op(const double2* A, int64_t lda, int64_t n, int64_t nrhs, const double2* w, double2* u,
                     hipStream_t s) {
  std::vector<GemmDesc> d{gemm(A, lda, OP_N, w, n, OP_T, u, n, n, nrhs, n)};
  d[0].transC = 1;
  zgemm_batched(d, s);
}

}  // namespace cbfm

using namespace cbfm;

extern "C" cbfm_status cbfm_solve(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, const void* Zr_v, int64_t ldz,
                                  const double* inc, int64_t nrhs, const cbfm_solver_params* prm, void* j_dev,
                                  int32_t* iters, double* relres, const double* dirs, int64_t ndir, double* rcs,
                                  void* stream) {
  cbfm_status noconv = CBFM_OK;
  cbfm_status st = guarded([&] {
    CBFM_REQUIRE(m && c && Zr_v && inc && prm, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(c->mesh == m, CBFM_E_STATE, "CBF set belongs to another mesh");
    CBFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, CBFM_E_ARG, "nrhs out of range");
    CBFM_REQUIRE(ldz >= 2 * c->NL, CBFM_E_ARG, "ldz < N_CBF");
    CBFM_REQUIRE(prm->tol > 0 && prm->max_iter >= 1 && prm->restart >= 1, CBFM_E_ARG, "bad solver parameters");
    CBFM_REQUIRE(dirs == nullptr || ndir >= 1, CBFM_E_ARG, "ndir must be >= 1 with dirs");
    const Media md = make_media(med);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MeshHost& h = m->h;
    const int64_t ne = h.ne, NL = c->NL, n = 2 * NL, nb = h.nblocks;
    const double2* Zr = static_cast<const double2*>(Zr_v);
    const bool use_cmp = prm->use_cmp != 0;
    const int64_t mres = std::min<int64_t>(prm->restart, std::max<int64_t>(prm->max_iter, 1));
    // ---- right-hand sides and their projection
    Scratch dinc(nrhs * 6 * sizeof(double), s);
    CBFM_HIP(hipMemcpyAsync(dinc.p, inc, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, s));
    Scratch v(nrhs * 2 * ne * sizeof(double2), s), vint(nrhs * 2 * ne * sizeof(double2), s);
    rhs_launch(m, md, med->eta0, dinc.as<double>(), nrhs, v.p, s);
    hipLaunchKernelGGL(permute_kernel, grid2(ne, nrhs), dim3(256), 0, s, v.as<double2>(), vint.as<double2>(),
                       m->perm.as<int32_t>(), ne, nrhs, 1);
    Scratch b(nrhs * n * sizeof(double2), s);
    {
      std::vector<GemmDesc> ds;
      for (int a = 0; a < nb; ++a) {
        const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], r0 = h.cell_off[a];
        // [v_r]_J-part = (C^J_a)^H v^E_a,  [v_r]_M-part = (C^M_a)^H v^H_a  (per vector: v . conj(C))
        ds.push_back(gemm(vint.as<double2>() + r0, 2 * ne, OP_N, c->CJ.as<double2>() + c->coff[a], c->L[a], OP_R,
                          b.as<double2>() + c->off[a], n, nrhs, c->L[a], Na));
        ds.push_back(gemm(vint.as<double2>() + ne + r0, 2 * ne, OP_N, c->CM.as<double2>() + c->coff[a], c->L[a], OP_R,
                          b.as<double2>() + NL + c->off[a], n, nrhs, c->L[a], Na));
      }
      zgemm_batched(ds, s);
    }
    // ---- operator: right-preconditioned A = Z_r (G^CBF)^{-1}, formed once,
    // with (G^CBF)^{-1} = blkdiag(-(B^{-1})^H, B^{-1})
    const double2* Aop = Zr;
    int64_t lda = ldz;
    Scratch Ap(use_cmp ? n * n * sizeof(double2) : 0, s);
    if (use_cmp) {
      const double2* Bi = cmp_inverse(c, s);
      std::vector<GemmDesc> ds{gemm(Zr, ldz, OP_N, Bi, NL, OP_C, Ap.as<double2>(), n, n, NL, NL, -1.0),
                               gemm(Zr + NL, ldz, OP_N, Bi, NL, OP_N, Ap.as<double2>() + NL, n, n, NL, NL)};
      zgemm_batched(ds, s);
      Aop = Ap.as<double2>();
      lda = n;
    }
    // ---- GMRES state
    Scratch V((mres + 1) * nrhs * n * sizeof(double2), s);
    Scratch x(nrhs * n * sizeof(double2), s), u(nrhs * n * sizeof(double2), s);
    const int np = (int)((n + 255) / 256);  // partial norm sums per vector
    Scratch Hs(nrhs * (mres + 1) * mres * sizeof(double2), s), csb(nrhs * mres * sizeof(double2), s),
        snb(nrhs * mres * sizeof(double2), s), gb(nrhs * (mres + 1) * sizeof(double2), s),
        hcol((mres + 2) * nrhs * sizeof(double2), s), h2((mres + 1) * nrhs * sizeof(double2), s),
        dbl(3 * nrhs * sizeof(double), s), ints(3 * nrhs * sizeof(int32_t), s), part(nrhs * np * sizeof(double), s),
        mask2(nrhs * sizeof(int32_t), s);
    GmresState gs{Hs.as<double2>(), csb.as<double2>(), snb.as<double2>(), gb.as<double2>(), hcol.as<double2>(),
                  dbl.as<double>(), dbl.as<double>() + nrhs, dbl.as<double>() + 2 * nrhs, ints.as<int32_t>(),
                  ints.as<int32_t>() + nrhs, ints.as<int32_t>() + 2 * nrhs};
    const int64_t vstride = nrhs * n;
    const dim3 g1((unsigned)((nrhs + 63) / 64)), b1(64), g4((unsigned)((nrhs + 3) / 4));
    CBFM_HIP(hipMemsetAsync(x.p, 0, nrhs * n * sizeof(double2), s));
    CBFM_HIP(hipMemsetAsync(gs.its, 0, nrhs * sizeof(int32_t), s));
    hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, b.as<double2>(), n, gs.bnorm, nullptr);
    std::vector<int32_t> its(nrhs, 0);
    std::vector<double> res(nrhs, 1.0);
    int64_t total = 0;
    const double tol = prm->tol;
    // Convergence flags go to pinned host memory every few iterations and are
    // read one check later, so the host never waits for the device inside a
    // cycle; iterations queued after the last right-hand side converged do
    // nothing (every kernel skips inactive right-hand sides).
    const int check_every = 4;
    PinnedFlags flags(nrhs);
    auto all_done = [&](const int32_t* a) {
      return std::none_of(a, a + nrhs, [](int32_t v) { return v != 0; });
    };
    // u = A v_j for every Krylov index j, descriptors uploaded once
    std::vector<std::vector<GemmDesc>> mv(mres);
    for (int64_t j = 0; j < mres; ++j) {
      GemmDesc d = gemm(Aop, lda, OP_N, V.as<double2>() + j * vstride, n, OP_T, u.as<double2>(), n, n, nrhs, n);
      d.transC = 1;
      mv[j].push_back(d);
    }
    const GemmPlan matvec(mv, s);
    for (;;) {
      // r = b - A x  (x = 0 on the first cycle)
      double2* r = u.as<double2>();
      if (total == 0) {
        CBFM_HIP(hipMemcpyAsync(r, b.p, nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
      } else {
        apply_op(Aop, lda, n, nrhs, x.as<double2>(), r, s);
        hipLaunchKernelGGL(sub_from_kernel, dim3((unsigned)((nrhs * n + 255) / 256)), dim3(256), 0, s, b.as<double2>(), r,
                           nrhs * n);
      }
      hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, r, n, gs.nrm, nullptr);
      hipLaunchKernelGGL(cycle_init_kernel, g1, b1, 0, s, gs, mres, nrhs, tol);
      hipLaunchKernelGGL(scale_kernel, grid2(n, nrhs), dim3(256), 0, s, r, V.as<double2>(), n, gs.nrm);
      if (all_done(flags.sync_read(gs.active, s)) || total >= prm->max_iter) break;
      int pending = 0;  // flag copies queued in this cycle
      for (int64_t j = 0; j < mres && total < prm->max_iter; ++j) {
        double2* Vn = V.as<double2>() + (j + 1) * vstride;
        matvec.launch((size_t)j, s);
        // classical Gram-Schmidt; a second pass where the first removed most
        // of the vector (the Hessenberg column is the sum of the passes)
        hipLaunchKernelGGL(dots_kernel, dim3((unsigned)(((j + 2) * nrhs + 3) / 4)), dim3(256), 0, s, V.as<double2>(),
                           vstride, u.as<double2>(), n, nrhs, j + 1, 1, gs.active, gs.hcol);
        hipLaunchKernelGGL(orth_update_kernel, grid2(n, nrhs), dim3(256), 0, s, V.as<double2>(), vstride,
                           u.as<double2>(), n, j + 1, nrhs, gs.active, gs.hcol, part.as<double>(), mask2.as<int32_t>(),
                           nullptr);
        hipLaunchKernelGGL(dots_kernel, dim3((unsigned)(((j + 1) * nrhs + 3) / 4)), dim3(256), 0, s, V.as<double2>(),
                           vstride, u.as<double2>(), n, nrhs, j + 1, 0, mask2.as<int32_t>(), h2.as<double2>());
        hipLaunchKernelGGL(orth_update_kernel, grid2(n, nrhs), dim3(256), 0, s, V.as<double2>(), vstride,
                           u.as<double2>(), n, j + 1, nrhs, mask2.as<int32_t>(), h2.as<double2>(), part.as<double>(),
                           nullptr, gs.hcol);
        hipLaunchKernelGGL(normalize_kernel, grid2(n, nrhs), dim3(256), 0, s, u.as<double2>(), Vn, n, part.as<double>(),
                           np, gs.nrm, gs.active);
        hipLaunchKernelGGL(givens_kernel, g4, dim3(256), 0, s, gs, mres, j, nrhs, tol);
        CBFM_HIP(hipGetLastError());
        ++total;
        if ((j + 1) % check_every == 0) {
          if (pending > 0 && all_done(flags.wait())) break;
          flags.post(gs.active, s);
          ++pending;
        }
      }
      hipLaunchKernelGGL(backsolve_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, gs, mres, nrhs);
      hipLaunchKernelGGL(x_update_kernel, grid2(n, nrhs), dim3(256), 0, s, gs, V.as<double2>(), vstride, x.as<double2>(),
                         n, nrhs);
      CBFM_HIP(hipGetLastError());
      if (total >= prm->max_iter) break;
    }
    CBFM_HIP(hipMemcpyAsync(its.data(), gs.its, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    // true relative residual of the preconditioned system
    {
      double2* r = u.as<double2>();
      apply_op(Aop, lda, n, nrhs, x.as<double2>(), r, s);
      hipLaunchKernelGGL(sub_from_kernel, dim3((unsigned)((nrhs * n + 255) / 256)), dim3(256), 0, s, b.as<double2>(), r,
                         nrhs * n);
      hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, r, n, gs.nrm, nullptr);
      std::vector<double> rn(nrhs), bn(nrhs);
      CBFM_HIP(hipMemcpyAsync(rn.data(), gs.nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      CBFM_HIP(hipMemcpyAsync(bn.data(), gs.bnorm, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      CBFM_HIP(hipStreamSynchronize(s));
      for (int64_t q = 0; q < nrhs; ++q) {
        res[q] = bn[q] > 0 ? rn[q] / bn[q] : 0.0;
        if (res[q] > tol * 10.0) noconv = CBFM_E_NOCONV;
      }
    }
    // j_CBF = G^{-1} x ; j = C^MJ j_CBF
    double2* jc = x.as<double2>();
    if (use_cmp) cmp_apply_dev(c, nrhs, jc, s);
    Scratch jint(nrhs * 2 * ne * sizeof(double2), s), jout(nrhs * 2 * ne * sizeof(double2), s);
    {
      std::vector<GemmDesc> ds;
      for (int a = 0; a < nb; ++a) {
        const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], r0 = h.cell_off[a];
        // alpha^M_a = C^M_a beta^M_a, alpha^J_a = C^J_a beta^J_a  (per vector: beta . C^T)
        ds.push_back(gemm(jc + c->off[a], n, OP_N, c->CM.as<double2>() + c->coff[a], c->L[a], OP_T,
                          jint.as<double2>() + r0, 2 * ne, nrhs, Na, c->L[a]));
        ds.push_back(gemm(jc + NL + c->off[a], n, OP_N, c->CJ.as<double2>() + c->coff[a], c->L[a], OP_T,
                          jint.as<double2>() + ne + r0, 2 * ne, nrhs, Na, c->L[a]));
      }
      zgemm_batched(ds, s);
    }
    double2* jfinal = j_dev ? static_cast<double2*>(j_dev) : jout.as<double2>();
    hipLaunchKernelGGL(permute_kernel, grid2(ne, nrhs), dim3(256), 0, s, jint.as<double2>(), jfinal,
                       m->perm.as<int32_t>(), ne, nrhs, 0);
    CBFM_HIP(hipGetLastError());
    // ---- RCS
    if (rcs) {
      const int64_t nd = dirs ? ndir : 1;
      std::vector<double> hd(nrhs * nd * 3), hp;
      if (dirs) {
        for (int64_t q = 0; q < nrhs; ++q) std::memcpy(&hd[q * nd * 3], dirs, nd * 3 * sizeof(double));
      } else {
        hp.resize(nrhs * 3);
        for (int64_t q = 0; q < nrhs; ++q)
          for (int x3 = 0; x3 < 3; ++x3) {
            hd[q * 3 + x3] = -inc[q * 6 + x3];
            hp[q * 3 + x3] = inc[q * 6 + 3 + x3];
          }
      }
      Scratch ddir(hd.size() * sizeof(double), s), dpol(hp.size() * sizeof(double), s),
          dsig(nrhs * nd * sizeof(double), s);
      CBFM_HIP(hipMemcpyAsync(ddir.p, hd.data(), hd.size() * sizeof(double), hipMemcpyHostToDevice, s));
      if (!hp.empty()) CBFM_HIP(hipMemcpyAsync(dpol.p, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, s));
      FarArgs fa{};
      fa.xyz9 = m->tri_xyz.as<double>();
      fa.tri_edge = m->tri_edge.as<int32_t>();
      fa.c64 = m->c64.as<double>();
      fa.nt = h.nt;
      fa.ne = ne;
      const double s15 = std::sqrt(15.0);
      const double qa = (6.0 - s15) / 21.0, qb = (6.0 + s15) / 21.0;
      const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
      const double Bq[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {1 - 2 * qa, qa, qa}, {qa, 1 - 2 * qa, qa}, {qa, qa, 1 - 2 * qa},
                               {1 - 2 * qb, qb, qb},        {qb, 1 - 2 * qb, qb}, {qb, qb, 1 - 2 * qb}};
      const double Wq[7] = {9.0 / 40.0, wa, wa, wa, wb, wb, wb};
      std::memcpy(fa.bary, Bq, sizeof(Bq));
      std::memcpy(fa.w, Wq, sizeof(Wq));
      fa.k0 = med->k0;
      fa.eta0 = med->eta0;
      hipLaunchKernelGGL(farfield_kernel, dim3((unsigned)nd, (unsigned)nrhs), dim3(256), 0, s, fa, jfinal, ddir.as<double>(),
                         hp.empty() ? nullptr : dpol.as<double>(), nd, dsig.as<double>());
      CBFM_HIP(hipGetLastError());
      CBFM_HIP(hipMemcpyAsync(rcs, dsig.p, nrhs * nd * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    CBFM_HIP(hipStreamSynchronize(s));
    if (iters) std::memcpy(iters, its.data(), nrhs * sizeof(int32_t));
    if (relres) std::memcpy(relres, res.data(), nrhs * sizeof(double));
    if (noconv != CBFM_OK) set_error("GMRES did not reach the tolerance for every right-hand side");
  });
  return st != CBFM_OK ? st : noconv;
}
