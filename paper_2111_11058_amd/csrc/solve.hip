// Reduced solve and RCS (paper Sec. III-C outer/inner CBFM equations and
// the current reconstruction; monostatic RCS after Knott).
//
//   v_r = (C^JM)^H v                   (tested incident fields, projected)
//   GMRES on  Z_r (G^CBF)^{-1} y = v_r, x0 = 0, restarted   (right precond.)
//   j_CBF = (G^CBF)^{-1} y,   j = C^MJ j_CBF
//   sigma = k0^2 / (4 pi) |eta0 N_perp - rhat x L|^2
//
// GMRES runs on the device for all right-hand sides at once, each with its
// own Krylov space (Saad's GMRES; classical Gram-Schmidt with delayed
// re-orthogonalisation; complex Givens rotations).  Matrix-vector products
// are matrix-core GEMMs over all right-hand sides; the Hessenberg updates
// run one wavefront per right-hand side.  The host reads the convergence
// flags every few iterations, one read behind.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <type_traits>

#include "cbf.h"
#include "gemm.h"
#include "solve.h"

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

// Krylov vectors are stored as complex double (plain form) or complex
// float (the basis of the compressed-basis form; basis and work vector of
// the mixed form's inner solves); arithmetic is always double.
__device__ inline double2 ld2(const double2* p) { return *p; }
__device__ inline double2 ld2(const float2* p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}
__device__ inline void st2(double2* p, double2 v) { *p = v; }
__device__ inline void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
// v as st2 leaves it in storage of the pointer's type
__device__ inline double2 stored2(const double2*, double2 v) { return v; }
__device__ inline double2 stored2(const float2*, double2 v) {
  return make_double2((double)(float)v.x, (double)(float)v.y);
}

__device__ inline double2 cconjmul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// x moved across the lanes of each row of 16 by a DPP pattern.
template <int CTRL>
__device__ inline double dpp_double(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront as a butterfly: every lane ends with
// the same bits.
__device__ inline double wave_sum(double x) {
  x += dpp_double<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_double<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_double<0x141>(x);  // row_half_mirror
  x += dpp_double<0x140>(x);  // row_mirror
  x += __shfl_xor(x, 16, 64);
  x += __shfl_xor(x, 32, 64);
  return x;
}

// nrm[c] = ||u[c]|| (one block of 256 per vector); skipped for inactive vectors
__global__ void __launch_bounds__(256) norm_kernel(const double2* __restrict__ u, int64_t n, double* __restrict__ nrm,
                                                   const int32_t* __restrict__ active) {
  const int64_t c = blockIdx.x;
  if (active && !active[c]) return;
  double s = 0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const double2 a = u[c * n + k];
    s += a.x * a.x + a.y * a.y;
  }
  s = wave_sum(s);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) nrm[c] = sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
}

// out[c] = in[c] / nrm[c] (zero if nrm[c] == 0); with qd, also the stored
// value in double there
template <typename TV>
__global__ void scale_kernel(const double2* __restrict__ in, TV* __restrict__ out, int64_t n,
                             const double* __restrict__ nrm, double2* __restrict__ qd = nullptr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (k >= n) return;
  const double s = nrm[c] > 0 ? 1.0 / nrm[c] : 0.0;
  const double2 a = in[c * n + k];
  const double2 v = make_double2(a.x * s, a.y * s);
  st2(out + c * n + k, v);
  if (qd) qd[c * n + k] = stored2(out, v);
}

// out = in rounded to complex float
__global__ void to_float_kernel(const double2* __restrict__ in, int64_t ldi, float2* __restrict__ out, int64_t ldo,
                                int64_t rows, int64_t cols) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (k >= cols || r >= rows) return;
  const double2 v = in[r * ldi + k];
  out[r * ldo + k] = make_float2((float)v.x, (float)v.y);
}

// r = b - r
__global__ void sub_from_kernel(const double2* __restrict__ b, double2* __restrict__ r, int64_t total) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  r[k] = make_double2(b[k].x - r[k].x, b[k].y - r[k].y);
}

// Arnoldi with classical Gram-Schmidt and delayed re-orthogonalisation (the
// second Gram-Schmidt pass of q_j is taken in iteration j, together with the
// first pass of w = A q_j, so that every iteration reads the Krylov basis
// twice instead of four times).  In iteration j, with q_0..q_{j-1} final
// and q_j orthogonalised once:
//   a_i = q_i^H q_j, b_i = q_i^H w (i < j), alpha = q_j^H q_j, beta = q_j^H w
//   gamma = sqrt(alpha - |a|^2),  q_j <- (q_j - Q a) / gamma
//   column j-1 of H (A q_{j-1} was expanded in the old q_j):
//       H[l][j-1] += H[j][j-1] a_l (l < j),  H[j][j-1] *= gamma
//   A q_j(new) = (w - A Q a) / gamma with A Q a = Q_{j+1} p, p = H a, so
//   h_l = (b_l - p_l) / gamma (l < j), h_j = ((beta - a^H b) / gamma - p_j) / gamma
//   w <- w / gamma - sum_{l <= j} c_l q_l,  c_l = p_l / gamma + h_l, that is
//   c_l = b_l / gamma (l < j) and c_j = (beta - a^H b) / gamma^2
//   H[l][j] = h_l, H[j+1][j] = ||w||, q_{j+1} = w / ||w||
// Column j-1 is final after the correction, so the Givens rotations and the
// convergence test run one iteration behind the matrix-vector product.
struct GmresState {
  double2* R;       // rotated Hessenberg (upper triangular), per right-hand side: column j, row i at
                    // [c * (m + 1) * m + j * (m + 1) + i]
  double2* H;       // Hessenberg matrix of the final basis, by rows: row l, column i at [(l * m + i) * nrhs + c]
  double2* cs;      // [c * m + i]
  double2* sn;      // [c * m + i]
  double2* g;       // [i * nrhs + c], i <= m
  double2* d1;      // [i * nrhs + c]: a_i, alpha at i = j
  double2* d2;      // [i * nrhs + c]: b_i, beta at i = j
  double2* ab;      // [c] a^H b
  double* gam;      // [c] gamma
  double* nrm;      // [c]
  double* bnorm;    // [c]
  double* res;      // [c] residual estimate / bnorm
  double* tgt;      // [c] residual norm at which this cycle stops
  int32_t* active;  // [c]
  int32_t* kc;      // [c] Krylov dimension reached in this cycle
  int32_t* its;     // [c] iterations spent (all cycles)
  // per right-hand side contiguous copies for the column step (one block
  // per right-hand side reads them along i): [c * (m + 1) + i]
  double2* d1t;     // a_i, alpha
  double2* d2t;     // b_i, beta
  double2* hc;      // the newest column of H (rows 0..j+1)
  int64_t ms;       // m + 1
  // few right-hand sides: the update pass splits the basis range of each
  // 128-row block over `split` blocks, which leave their sums (128 rows x
  // the two sums) in ws at [((c np + rb) split + part) 256 + 128 s + 64 r +
  // lane]; dcgs_finish_kernel adds them in part order and completes the
  // update
  int split;
  double2* ws;
};

// The end of the update of 128 rows of one right-hand side (one wavefront,
// RPL = 2 rows per lane) once s1 = sum a_l q_l and s2 = sum b_l q_l are
// known: q_j <- (q_j - s1) / gamma, w <- (w - s2) / gamma - c_j q_j, and
// the partial sum of |w|^2 of these rows.
template <typename TB, typename TW>
__device__ inline void finish_rows(TB* V, int64_t vstride, TW* w, int64_t n, int64_t nrhs, int64_t j, int64_t c,
                                   int64_t rb, int np, const GmresState& st, const double2 (&s1)[2],
                                   const double2 (&s2)[2], double* part, int lane) {
  const double ig = 1.0 / st.gam[c];
  const double2 beta = st.d2[j * nrhs + c], ab = st.ab[c];
  const double2 cj = cscale(make_double2(beta.x - ab.x, beta.y - ab.y), ig * ig);
  double q2 = 0;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int64_t k = (rb * 2 + r) * 64 + lane;
    if (k < n) {
      TB* qj = V + j * vstride + c * n + k;
      const double2 qo = ld2(qj);
      const double2 qn = stored2(qj, cscale(make_double2(qo.x - s1[r].x, qo.y - s1[r].y), ig));
      st2(qj, qn);
      const double2 wo = ld2(w + c * n + k);
      const double2 t = cmul(cj, qn);
      const double2 wn = make_double2((wo.x - s2[r].x) * ig - t.x, (wo.y - s2[r].y) * ig - t.y);
      st2(w + c * n + k, wn);
      q2 += wn.x * wn.x + wn.y * wn.y;
    }
  }
  q2 = wave_sum(q2);
  if (lane == 0) part[c * np + rb] = q2;
}

// Start a cycle: g = beta e1, active = beta/bnorm > tol, kc = 0; the cycle
// stops at the residual norm max(tol bnorm, inner beta) (inner = 0: at tol;
// inner > 0: the relative reduction asked of an inner solve).
__global__ void cycle_init_kernel(GmresState st, int64_t m, int64_t nrhs, double tol, double inner) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double beta = st.nrm[c];
  for (int64_t i = 0; i <= m; ++i) st.g[i * nrhs + c] = make_double2(0, 0);
  st.g[c] = make_double2(beta, 0);
  const double r = st.bnorm[c] > 0 ? beta / st.bnorm[c] : 0.0;
  st.res[c] = r;
  st.active[c] = r > tol ? 1 : 0;
  st.tgt[c] = fmax(tol * st.bnorm[c], inner * beta);
  st.kc[c] = 0;
}

// d1[i] = q_i^H q_j and d2[i] = q_i^H w for i <= j: one block of four
// wavefronts per right-hand side and run of VPB = 4 basis vectors; the
// threads take every 256th row, the loads of all VPB vectors of a row go
// out together, and the wavefronts are summed through LDS in a fixed order.
// (For a float basis, runs of 8 vectors measured slower: half the blocks at
// 4 instead of 7 wavefronts per SIMD.)
template <typename TB, typename TW, bool UNR, int VPB = 4>
__global__ void __launch_bounds__(256) dots2_kernel(const TB* __restrict__ V, int64_t vstride,
                                                    const TW* __restrict__ w, int64_t n, int64_t nrhs, int64_t j,
                                                    GmresState st, const int64_t* __restrict__ jp) {
  static_assert(!UNR || VPB == 4, "the unrolled rows take four vectors");
  if (jp) j = *jp;  // iteration index from the device (graph replays)
  const int64_t id = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t runs = (j + VPB) / VPB;
  if (id >= runs * nrhs) return;  // uniform over the block
  const int64_t run = id / nrhs, c = id % nrhs;
  if (!st.active[c]) return;
  const int64_t i0 = run * VPB;
  const int cnt = (int)std::min<int64_t>(VPB, j + 1 - i0);
  const TB* qj = V + j * vstride + c * n;
  const TW* wc = w + c * n;
  const TB* qi = V + i0 * vstride + c * n;
  double2 s1[VPB], s2[VPB];
#pragma unroll
  for (int t = 0; t < VPB; ++t) s1[t] = s2[t] = make_double2(0, 0);
  int64_t k = threadIdx.x;
  // UNR: four rows per lane at a time, their loads issued together (the
  // sums still take the rows in order), for long vectors and few blocks;
  // it needs more registers, which would cost occupancy otherwise
  for (; UNR && k + 768 < n; k += 1024) {
    double2 x[4], y[4], v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = ld2(qj + k + 256 * u);
      y[u] = ld2(wc + k + 256 * u);
#pragma unroll
      for (int t = 0; t < 4; ++t) v[u][t] = ld2(qi + (t < cnt ? t : 0) * vstride + k + 256 * u);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        s1[t] = cadd(s1[t], cconjmul(v[u][t], x[u]));
        s2[t] = cadd(s2[t], cconjmul(v[u][t], y[u]));
      }
  }
  for (; k < n; k += 256) {
    const double2 x = ld2(qj + k), y = ld2(wc + k);
    double2 v[VPB];
#pragma unroll
    for (int t = 0; t < VPB; ++t) v[t] = ld2(qi + (t < cnt ? t : 0) * vstride + k);  // vectors past j: discarded
#pragma unroll
    for (int t = 0; t < VPB; ++t) {
      s1[t] = cadd(s1[t], cconjmul(v[t], x));
      s2[t] = cadd(s2[t], cconjmul(v[t], y));
    }
  }
  __shared__ double sh[4][VPB][4];
#pragma unroll
  for (int t = 0; t < VPB; ++t) {
    const double r0 = wave_sum(s1[t].x), r1 = wave_sum(s1[t].y), r2 = wave_sum(s2[t].x), r3 = wave_sum(s2[t].y);
    if (lane == 0) {
      sh[wv][t][0] = r0;
      sh[wv][t][1] = r1;
      sh[wv][t][2] = r2;
      sh[wv][t][3] = r3;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < cnt) {
    double r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = (sh[0][t][q] + sh[1][t][q]) + (sh[2][t][q] + sh[3][t][q]);
    const double2 v1 = make_double2(r[0], r[1]), v2 = make_double2(r[2], r[3]);
    st.d1[(i0 + t) * nrhs + c] = v1;
    st.d2[(i0 + t) * nrhs + c] = v2;
    st.d1t[c * st.ms + i0 + t] = v1;
    st.d2t[c * st.ms + i0 + t] = v2;
  }
}

// Per right-hand side (one block of 256 threads each): gamma and a^H b,
// then column jc = j - 1 made final (corrected for the new q_j unless
// correct == 0, the end of a cycle, when it is taken as it stands) and
// reduced by the Givens rotations; the new rotation updates g and the
// convergence test.
// Rotation i maps (a_i, h_{i+1}) to (c_i a_i + s_i h_{i+1}, a_{i+1}) with
// a_{i+1} = -conj(s_i) a_i + conj(c_i) h_{i+1}, a_0 = h_0: the carried a_i
// follow an affine recurrence, so each thread composes the maps of a
// contiguous run of rotations (at most four up to 1024 columns), a scan over
// the block gives every run its incoming a_i, and the runs are then replayed
// in parallel.  The kernel is bound by memory latency: every load a thread
// needs is issued before its first wait (up to 1024 columns), so it waits
// on memory about once instead of once per step.
__global__ void __launch_bounds__(256) column_kernel(GmresState st, int64_t m, int64_t j, int64_t nrhs,
                                                      int correct, const int64_t* __restrict__ jp) {
  if (jp) j = *jp;
  const int64_t c = (int64_t)blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (c >= nrhs) return;
  // this right-hand side's contiguous vectors
  const double2* d1 = st.d1t + c * st.ms;
  const double2* d2 = st.d2t + c * st.ms;
  const double2* hcol = st.hc + c * st.ms;
  double2* sn = st.sn + c * m;
  double2* cs = st.cs + c * m;
  __shared__ double red[4][3];
  __shared__ double2 tot[4][2];     // (P, Q) of each wavefront's runs
  __shared__ double2 incl[256][2];  // (P, Q) of runs 0..t
  __shared__ double2 afin;
  constexpr int KR = 4;
  const int64_t jc = j > 0 ? j - 1 : 0, col = jc * (m + 1);
  const int64_t K = (jc + 255) / 256;
  const int64_t i0 = std::min<int64_t>(jc, t * K), i1 = std::min<int64_t>(jc, i0 + K);
  // ---- loads (indices clamped to valid entries; the unused ones discarded)
  double2 da[KR], db[KR];  // a_l, b_l of iteration j for l = t + 256 u
#pragma unroll
  for (int u = 0; u < KR; ++u) {
    const int64_t l = t + 256 * u < j ? t + 256 * u : 0;
    da[u] = d1[l];
    db[u] = d2[l];
  }
  const double alpha = d1[j].x;
  const double2 hs = hcol[jc + 1];  // H[jc+1][jc], real
  const double2 h0 = hcol[0], a00 = d1[0], gj = st.g[jc * nrhs + c];
  const double tgt = st.tgt[c], bnorm = st.bnorm[c];
  double2 sv[KR], cv[KR], bv[KR];  // first KR rotations of this thread's run
#pragma unroll
  for (int u = 0; u < KR; ++u) {
    const int64_t i = std::max<int64_t>(0, std::min<int64_t>(i0 + u, i1 - 1));
    sv[u] = sn[i];
    cv[u] = cs[i];
    bv[u] = hcol[i + 1];
    if (correct) bv[u] = cadd(bv[u], cmul(hs, d1[i + 1]));
  }
  // (the loads above are issued for converged right-hand sides too: the
  // test comes after them so that it does not delay them)
  if (!st.active[c]) return;  // uniform over the block
  // ---- gamma and a^H b
  double gam = 1.0;
  bool breakdown = false;
  if (correct) {
    double aa = 0;
    double2 ab = make_double2(0, 0);
#pragma unroll
    for (int u = 0; u < KR; ++u)
      if (t + 256 * u < j) {
        aa += da[u].x * da[u].x + da[u].y * da[u].y;
        ab = cadd(ab, cconjmul(da[u], db[u]));
      }
    for (int64_t l = t + 256 * KR; l < j; l += 256) {
      const double2 a = d1[l];
      aa += a.x * a.x + a.y * a.y;
      ab = cadd(ab, cconjmul(a, d2[l]));
    }
    aa = wave_sum(aa);
    ab = make_double2(wave_sum(ab.x), wave_sum(ab.y));
    if (lane == 0) {
      red[wv][0] = aa;
      red[wv][1] = ab.x;
      red[wv][2] = ab.y;
    }
    __syncthreads();
    aa = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    ab = make_double2((red[0][1] + red[1][1]) + (red[2][1] + red[3][1]),
                      (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]));
    const double g2 = alpha - aa;
    // q_j nearly inside the span of q_0..q_{j-1}: the Krylov space is
    // (numerically) invariant, taken as a breakdown
    breakdown = !(g2 > 0.25 * alpha);
    gam = breakdown ? 1.0 : sqrt(g2);
    if (t == 0) {
      st.gam[c] = gam;
      st.ab[c] = ab;
    }
  }
  if (j == 0) return;
  const double hsub = correct ? (breakdown ? 0.0 : hs.x * gam) : hs.x;
  // ---- compose the maps of this thread's run
  double2 P = make_double2(1, 0), Q = make_double2(0, 0);
  for (int64_t ib = i0; ib < i1; ib += KR) {
    double2 s2[KR], c2[KR], b2[KR];
#pragma unroll
    for (int u = 0; u < KR; ++u) {
      s2[u] = sv[u];
      c2[u] = cv[u];
      b2[u] = bv[u];
    }
    if (ib != i0) {  // past the first KR rotations (more than 1024 columns)
#pragma unroll
      for (int u = 0; u < KR; ++u) {
        const int64_t i = std::min<int64_t>(ib + u, i1 - 1);
        s2[u] = sn[i];
        c2[u] = cs[i];
        b2[u] = hcol[i + 1];
        if (correct) b2[u] = cadd(b2[u], cmul(hs, d1[i + 1]));
      }
    }
#pragma unroll
    for (int u = 0; u < KR; ++u) {
      if (ib + u >= i1) break;
      if (correct) st.H[((ib + u + 1) * m + jc) * nrhs + c] = b2[u];
      const double2 Pi = make_double2(-s2[u].x, s2[u].y);  // -conj(s_i)
      Q = cadd(cmul(Pi, Q), cmul(make_double2(c2[u].x, -c2[u].y), b2[u]));
      P = cmul(Pi, P);
    }
  }
  // ---- inclusive scan over the wavefront, then over the wavefronts in
  // order: afterwards (P, Q) maps a_0 to the carry leaving run t
  for (int off = 1; off < 64; off <<= 1) {
    const double2 Po = make_double2(__shfl_up(P.x, off, 64), __shfl_up(P.y, off, 64));
    const double2 Qo = make_double2(__shfl_up(Q.x, off, 64), __shfl_up(Q.y, off, 64));
    if (lane >= off) {
      Q = cadd(cmul(P, Qo), Q);
      P = cmul(P, Po);
    }
  }
  if (lane == 63) {
    tot[wv][0] = P;
    tot[wv][1] = Q;
  }
  __syncthreads();
  double2 Pp = make_double2(1, 0), Qp = make_double2(0, 0);
  for (int v = 0; v < wv; ++v) {
    Qp = cadd(cmul(tot[v][0], Qp), tot[v][1]);
    Pp = cmul(tot[v][0], Pp);
  }
  Q = cadd(cmul(P, Qp), Q);
  P = cmul(P, Pp);
  incl[t][0] = P;
  incl[t][1] = Q;
  __syncthreads();
  const double2 a0 = correct ? cadd(h0, cmul(hs, a00)) : h0;
  double2 a = t == 0 ? a0 : cadd(cmul(incl[t - 1][0], a0), incl[t - 1][1]);
  // ---- replay the run: rotated column entries
  for (int64_t ib = i0; ib < i1; ib += KR) {
    double2 s2[KR], c2[KR], b2[KR];
#pragma unroll
    for (int u = 0; u < KR; ++u) {
      s2[u] = sv[u];
      c2[u] = cv[u];
      b2[u] = bv[u];
    }
    if (ib != i0) {  // this thread stored the final H[i+1][jc] above
#pragma unroll
      for (int u = 0; u < KR; ++u) {
        const int64_t i = std::min<int64_t>(ib + u, i1 - 1);
        s2[u] = sn[i];
        c2[u] = cs[i];
        b2[u] = st.H[((i + 1) * m + jc) * nrhs + c];
      }
    }
#pragma unroll
    for (int u = 0; u < KR; ++u) {
      if (ib + u >= i1) break;
      st.R[c * (m + 1) * m + col + ib + u] = cadd(cmul(c2[u], a), cmul(s2[u], b2[u]));
      a = cadd(cmul(make_double2(-s2[u].x, s2[u].y), a), cmul(make_double2(c2[u].x, -c2[u].y), b2[u]));
    }
  }
  const int last = jc == 0 ? 0 : (int)((jc - 1) / K);  // thread that ends with a_jc
  if (t == last) afin = a;
  __syncthreads();
  if (t != 0) return;
  a = afin;
  if (correct) {
    st.H[jc * nrhs + c] = a0;
    st.H[((jc + 1) * m + jc) * nrhs + c] = make_double2(hsub, 0);
  }
  const double den = sqrt(a.x * a.x + a.y * a.y + hsub * hsub);
  double2 cc = make_double2(1, 0), ss = make_double2(0, 0);
  if (den > 0) {
    cc = make_double2(a.x / den, -a.y / den);  // conj(a)/den
    ss = make_double2(hsub / den, 0.0);        // conj(h)/den, h real
  }
  cs[jc] = cc;
  sn[jc] = ss;
  st.R[c * (m + 1) * m + col + jc] = make_double2(den, 0);
  // g[jc+1] = -conj(s) g[jc];  g[jc] = c g[jc]
  const double2 gn = make_double2(-(ss.x * gj.x + ss.y * gj.y), -(ss.x * gj.y - ss.y * gj.x));
  st.g[(jc + 1) * nrhs + c] = gn;
  st.g[jc * nrhs + c] = cmul(cc, gj);
  const double ra = sqrt(gn.x * gn.x + gn.y * gn.y);
  st.res[c] = ra / bnorm;
  st.kc[c] = (int32_t)(jc + 1);
  st.its[c] += 1;
  if (ra <= tgt || den == 0.0 || breakdown) st.active[c] = 0;
}

// The update pass, with column j of H computed beside it.  With
// p_l = sum_i H[l][i] a_i over the final columns i < j (upper Hessenberg:
// i >= l - 1), h_l = (b_l - p_l) / gamma, h_j = ((beta - a^H b) / gamma -
// p_j) / gamma and c_l = p_l / gamma + h_l, the update coefficients reduce
// to c_l = b_l / gamma (l < j) and c_j = (beta - a^H b) / gamma^2, so the
// update does not wait for p:
//   q_j <- (q_j - sum_{i<j} a_i q_i) / gamma
//   w   <- (w - sum_{i<j} b_i q_i) / gamma - c_j q_j(new)
// Blocks [0, np nrhs split): eight wavefronts take 128 consecutive rows (two
// per lane) of one right-hand side, wavefront v summing over the basis
// vectors i = v mod 8 (with split > 1, part p of the row block over those
// with i / 8 = p mod split); wavefront 0 combines the partial sums in a
// fixed order and completes the update, storing the row block's sum of
// |w|^2 in part (with split > 1, dcgs_finish_kernel does this).
// Blocks from np nrhs split on: row l of column j; the lanes take up to 64
// right-hand sides and, when there are fewer, several column offsets each
// (added by a butterfly); the eight wavefronts take interleaved columns of
// the row (contiguous in H), four columns in flight each, summed in a fixed
// order.  These latency-bound blocks come last, where they fill
// the tail of the streaming; placed first they held CUs the update blocks
// needed, and cutting the rows into parts or running them as a separate
// launch or stream measured slower too.
template <typename TB, typename TW, bool SPLIT>
__global__ void __launch_bounds__(512) dcgs_update_kernel(TB* __restrict__ V, int64_t vstride,
                                                          TW* __restrict__ w, int64_t n, int64_t nrhs, int64_t m,
                                                          int64_t j, int np, GmresState st,
                                                          double* __restrict__ part, const int64_t* __restrict__ jp) {
  if (jp) j = *jp;
  // wv is uniform over the wavefront: the coefficient loads below go through scalar loads
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int S = SPLIT ? st.split : 1;
  const int64_t nub = (int64_t)np * nrhs * S;  // update blocks
  if ((int64_t)blockIdx.x >= nub) {
    __shared__ double2 shp[7][64];
    const int64_t hb = (int64_t)blockIdx.x - nub;
    const int64_t ng = (nrhs + 63) / 64;
    // lanes: cw right-hand sides (a power of two, at least nrhs when nrhs <
    // 64) times 64 / cw column offsets, so that few right-hand sides still
    // fill the wavefront; with 64 or more, one column offset per lane group
    int cw = 64;
    while (cw > 1 && cw / 2 >= nrhs) cw >>= 1;
    const int sub = 64 / cw, lc = lane & (cw - 1), li = lane / cw;
    const int64_t l = hb / ng, c = (hb % ng) * 64 + lc;
    if (l > j) return;  // graph replays launch the rows of the longest column
    const bool on = c < nrhs && st.active[c];
    const int64_t cc = on ? c : 0;  // idle lanes read valid entries and discard them
    const int64_t lo = l > 0 ? l - 1 : 0;
    const double2* Hl = st.H + l * m * nrhs + cc;  // column i at Hl[i * nrhs]: the row is contiguous
    const double2* a = st.d1 + cc;
    double2 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = make_double2(0, 0);
    const int64_t istep = 8 * (int64_t)sub;  // column stride of one unrolled load
    for (int64_t ib = lo + wv * sub + li; ib < j; ib += 4 * istep) {
      double2 hv[4], av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = ib + istep * u < j ? ib + istep * u : ib;
        hv[u] = Hl[i * nrhs];
        av[u] = a[i * nrhs];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = ib + istep * u < j ? cadd(acc[u], cmul(hv[u], av[u])) : acc[u];
    }
    double2 p = cadd(cadd(acc[0], acc[1]), cadd(acc[2], acc[3]));
    for (int off = cw; off < 64; off <<= 1)  // the column offsets of one right-hand side
      p = make_double2(p.x + __shfl_xor(p.x, off, 64), p.y + __shfl_xor(p.y, off, 64));
    if (wv > 0) shp[wv - 1][lane] = p;
    __syncthreads();
    if (wv > 0 || !on || li != 0) return;
    for (int v = 0; v < 7; ++v) p = cadd(p, shp[v][lane]);
    const double ig = 1.0 / st.gam[c];
    const double2 b = st.d2[l * nrhs + c];
    double2 h;
    if (l < j) {
      h = cscale(make_double2(b.x - p.x, b.y - p.y), ig);
    } else {
      const double2 ab = st.ab[c];
      h = cscale(make_double2((b.x - ab.x) * ig - p.x, (b.y - ab.y) * ig - p.y), ig);
    }
    st.H[(l * m + j) * nrhs + c] = h;
    st.hc[c * st.ms + l] = h;
    return;
  }
  constexpr int RPL = 2;  // rows per lane (finish_rows takes two)
  const int part_id = (int)(blockIdx.x % S);
  const int64_t c = (int64_t)(blockIdx.x / S) / np, rb = (int64_t)(blockIdx.x / S) % np;
  if (c >= nrhs || !st.active[c]) return;  // uniform over the block
  const double2* d1 = st.d1;
  const double2* d2 = st.d2;
  double2 s1[RPL], s2[RPL];
  int64_t kk[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    s1[r] = s2[r] = make_double2(0, 0);
    const int64_t k = (rb * RPL + r) * 64 + lane;
    kk[r] = k < n ? k : 0;  // rows past n: a valid row, discarded
  }
  const TB* base = V + c * n;
  // this block's basis vectors: i = 8 (part + S t) + wavefront
  const int64_t istep = 8 * (int64_t)S;
  int64_t i = wv + 8 * (int64_t)part_id;
  // U basis vectors at a time (4; 8 for a float basis beside a double w,
  // the same bytes in flight, measured 201 -> 184 us on 4,224 rows x 32
  // right-hand sides): their loads go out together (the sums still take
  // the vectors in order)
  constexpr int U = sizeof(TB) < sizeof(TW) ? 8 : 4;
  for (; i + (U - 1) * istep < j; i += U * istep) {
    double2 a[U], b[U], v[U][RPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = d1[(i + istep * u) * nrhs + c];
      b[u] = d2[(i + istep * u) * nrhs + c];
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[u][r] = ld2(base + (i + istep * u) * vstride + kk[r]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        s1[r] = cadd(s1[r], cmul(a[u], v[u][r]));
        s2[r] = cadd(s2[r], cmul(b[u], v[u][r]));
      }
  }
  for (; i < j; i += istep) {
    const double2 a = d1[i * nrhs + c], b = d2[i * nrhs + c];
    double2 v[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) v[r] = ld2(base + i * vstride + kk[r]);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      s1[r] = cadd(s1[r], cmul(a, v[r]));
      s2[r] = cadd(s2[r], cmul(b, v[r]));
    }
  }
  __shared__ double2 sh[7][RPL][64][2];
  if (wv > 0) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      sh[wv - 1][r][lane][0] = s1[r];
      sh[wv - 1][r][lane][1] = s2[r];
    }
  }
  __syncthreads();
  if (wv > 0) return;
#pragma unroll
  for (int r = 0; r < RPL; ++r)
    for (int t = 0; t < 7; ++t) {
      s1[r] = cadd(s1[r], sh[t][r][lane][0]);
      s2[r] = cadd(s2[r], sh[t][r][lane][1]);
    }
  if (SPLIT) {  // dcgs_finish_kernel completes the update
    double2* mine = st.ws + (((c * np + rb) * S) + part_id) * 256;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      mine[64 * r + lane] = s1[r];
      mine[128 + 64 * r + lane] = s2[r];
    }
    return;
  }
  finish_rows(V, vstride, w, n, nrhs, j, c, rb, np, st, s1, s2, part, lane);
}

// The update of a split pass: one wavefront per 128-row block of a
// right-hand side adds the parts' sums in part order and completes it.
template <typename TB, typename TW>
__global__ void __launch_bounds__(64) dcgs_finish_kernel(TB* __restrict__ V, int64_t vstride, TW* __restrict__ w,
                                                          int64_t n, int64_t nrhs, int64_t j, int np, GmresState st,
                                                          double* __restrict__ part, const int64_t* __restrict__ jp) {
  if (jp) j = *jp;
  const int lane = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x / np, rb = (int64_t)blockIdx.x % np;
  if (c >= nrhs || !st.active[c]) return;
  const int S = st.split;
  const double2* sums = st.ws + (c * np + rb) * S * 256;
  double2 s1[2], s2[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    s1[r] = s2[r] = make_double2(0, 0);
    for (int q = 0; q < S; ++q) {
      s1[r] = cadd(s1[r], sums[q * 256 + 64 * r + lane]);
      s2[r] = cadd(s2[r], sums[q * 256 + 128 + 64 * r + lane]);
    }
  }
  finish_rows(V, vstride, w, n, nrhs, j, c, rb, np, st, s1, s2, part, lane);
}

// nu = sqrt(sum of the np partial sums of |w|^2); H[j+1][j] = nu and
// q_{j+1} = w / nu (zero if nu == 0), with qd also its stored value in
// double (the operand of the next matrix-vector product); only active
// right-hand sides.
template <typename TB, typename TW>
__global__ void normalize_kernel(const TW* __restrict__ w, TB* __restrict__ V, int64_t vstride, int64_t n,
                                 const double* __restrict__ part, int np, GmresState st, int64_t m, int64_t j,
                                 int64_t nrhs, const int64_t* __restrict__ jp, double2* __restrict__ qd) {
  if (jp) j = *jp;
  TB* out = V + (j + 1) * vstride;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (!st.active[c]) return;
  double q = 0;
  for (int b = 0; b < np; ++b) q += part[c * np + b];
  const double nu = sqrt(q);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st.H[((j + 1) * m + j) * nrhs + c] = make_double2(nu, 0);
    st.hc[c * st.ms + j + 1] = make_double2(nu, 0);
  }
  if (k >= n) return;
  const double sc = nu > 0 ? 1.0 / nu : 0.0;
  const double2 v = cscale(ld2(w + c * n + k), sc);
  st2(out + c * n + k, v);
  if (qd) qd[c * n + k] = stored2(out, v);
}

// Device-side iteration counter of graph replays, and the matrix-vector
// product's operand q_j taken from it.
__global__ void counter_kernel(int64_t* __restrict__ jp, int64_t value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *jp = add ? *jp + value : value;
}
template <typename D, typename TV>
__global__ void point_matvec_kernel(D* __restrict__ desc, const TV* V, int64_t vstride, const int64_t* __restrict__ jp) {
  if (threadIdx.x == 0 && blockIdx.x == 0) desc->B = V + (*jp) * vstride;
}

// y = R^{-1} g over the first kc[c] rows (R upper triangular), in place in
// g; one block per right-hand side.  Blocked back substitution: the
// triangle of the lowest 32 unsolved rows is copied to LDS and solved by one
// wavefront (the solved value broadcast across the lanes), then every row
// above it is updated by the block with all 32 loads of a row issued
// together, so the block waits on memory about twice per 32 rows instead of
// once per row.
__global__ void __launch_bounds__(256) backsolve_kernel(GmresState st, int64_t m, int64_t nrhs) {
  constexpr int BS = 32;
  const int64_t c = blockIdx.x;
  const int64_t k = st.kc[c];
  __shared__ double2 T[BS][BS + 1];  // T[r][q] = R[b0 + r][b0 + q], q >= r
  __shared__ double2 yb[BS];         // solved values of the block
  const int tid = threadIdx.x;
  const double2* Rc = st.R + c * (m + 1) * m;  // this right-hand side's R, column-major
  for (int64_t b1 = k; b1 > 0; b1 -= BS) {
    const int64_t b0 = b1 > BS ? b1 - BS : 0;
    const int nb = (int)(b1 - b0);
    for (int e = tid; e < nb * nb; e += 256) {
      const int q = e / nb, r = e % nb;  // consecutive threads: consecutive rows of column q
      if (q >= r) T[r][q] = Rc[(b0 + q) * (m + 1) + b0 + r];
    }
    __syncthreads();
    if (tid < 64) {
      const int lane = tid;
      double2 yl = lane < nb ? st.g[(b0 + lane) * nrhs + c] : make_double2(0, 0);
      for (int q = nb - 1; q >= 0; --q) {
        if (lane == q) {
          const double2 d = T[q][q];
          const double dd = d.x * d.x + d.y * d.y;
          yl = dd > 0 ? make_double2((yl.x * d.x + yl.y * d.y) / dd, (yl.y * d.x - yl.x * d.y) / dd)
                      : make_double2(0, 0);
        }
        const double2 yq = make_double2(__shfl(yl.x, q, 64), __shfl(yl.y, q, 64));
        if (lane < q) yl = make_double2(yl.x - (T[lane][q].x * yq.x - T[lane][q].y * yq.y),
                                        yl.y - (T[lane][q].x * yq.y + T[lane][q].y * yq.x));
      }
      if (lane < nb) {
        yb[lane] = yl;
        st.g[(b0 + lane) * nrhs + c] = yl;
      }
    }
    __syncthreads();
    for (int64_t t = tid; t < b0; t += 256) {
      double2 h[BS];
#pragma unroll
      for (int q = 0; q < BS; ++q) h[q] = Rc[(b0 + (q < nb ? q : 0)) * (m + 1) + t];
      double2 acc = make_double2(0, 0);
#pragma unroll
      for (int q = 0; q < BS; ++q)
        if (q < nb) acc = cadd(acc, cmul(h[q], yb[q]));
      double2* gt = st.g + t * nrhs + c;
      *gt = make_double2(gt->x - acc.x, gt->y - acc.y);
    }
    __syncthreads();
  }
}

// x[c] += sum_{i < kc[c]} y[i][c] V[i][c]: a block of eight wavefronts takes
// 128 consecutive rows (two per lane) of one right-hand side, wavefront v
// summing over the basis vectors i = v mod 8, combined in a fixed order.
template <typename TV>
__global__ void __launch_bounds__(512) x_update_kernel(GmresState st, const TV* __restrict__ V, int64_t vstride,
                                                       double2* __restrict__ x, int64_t n, int64_t nrhs, int np) {
  constexpr int RPL = 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = blockIdx.x / np, rb = blockIdx.x % np;
  if (c >= nrhs) return;
  const int64_t kc = st.kc[c];
  double2 acc[RPL];
  int64_t kk[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    acc[r] = make_double2(0, 0);
    const int64_t k = (rb * RPL + r) * 64 + lane;
    kk[r] = k < n ? k : 0;  // rows past n: a valid row, discarded
  }
  const TV* base = V + c * n;
  int64_t i = wv;
  // four basis vectors at a time: their loads go out together (the sums
  // still take the vectors in order)
  for (; i + 24 < kc; i += 32) {
    double2 a[4], v[4][RPL];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = st.g[(i + 8 * u) * nrhs + c];
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[u][r] = ld2(base + (i + 8 * u) * vstride + kk[r]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[r] = cadd(acc[r], cmul(a[u], v[u][r]));
  }
  for (; i < kc; i += 8) {
    const double2 a = st.g[i * nrhs + c];
    double2 v[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) v[r] = ld2(base + i * vstride + kk[r]);
#pragma unroll
    for (int r = 0; r < RPL; ++r) acc[r] = cadd(acc[r], cmul(a, v[r]));
  }
  __shared__ double2 sh[7][RPL][64];
  if (wv > 0) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) sh[wv - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (wv > 0) return;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    for (int t = 0; t < 7; ++t) acc[r] = cadd(acc[r], sh[t][r][lane]);
    const int64_t k = (rb * RPL + r) * 64 + lane;
    if (k < n) x[c * n + k] = cadd(x[c * n + k], acc[r]);
  }
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

static dim3 grid2(int64_t n, int64_t m) { return dim3((unsigned)((n + 255) / 256), (unsigned)m); }

// u = A w for row-stored vectors w (nrhs x n): u^T = A w^T.
static void apply_op(const double2* A, int64_t lda, int64_t n, int64_t nrhs, const double2* w, double2* u,
                     hipStream_t s) {
  std::vector<GemmDesc> d{gemm(A, lda, OP_N, w, n, OP_T, u, n, n, nrhs, n)};
  d[0].transC = 1;
  zgemm_batched(d, s);
}

// One GMRES cycle from the normalised residual in V[0]: up to mres Arnoldi
// iterations (the matrix-vector products by mv.launch(j)), the last column,
// the triangular solve and x += Q y.  total counts the iterations of all
// cycles against max_iter.  With a graph plan (dyn, its descriptor dyn_desc
// and the device counter jdev), chunks of four iterations are captured once
// into a HIP graph whose kernels read the iteration index from jdev, and
// the graph is replayed; the remaining iterations run as plain launches.
// The basis is stored as TB and the work vector w as TW.  With qd (a float
// basis beside a double w), every matrix-vector product reads its operand
// from qd, where the newest basis vector's stored value is kept in double.
template <typename TB, typename TW, typename MV>
static void run_cycle(const MV& mv, const MV* dyn, void* dyn_desc, int64_t* jdev, TB* V, TW* w, int64_t vstride,
                      int64_t n, int64_t nrhs, int64_t mres, int64_t max_iter, int64_t& total, GmresState gs,
                      double* part, int np, PinnedFlags& flags, double2* x, hipStream_t s, const TB* xb = nullptr,
                      double2* qd = nullptr) {
  const double vb = (double)sizeof(TB), wb = (double)sizeof(TW);
  const int check_every = 4;
  const int64_t ng = (nrhs + 63) / 64;
  auto all_done = [&](const int32_t* a) { return std::none_of(a, a + nrhs, [](int32_t v) { return v != 0; }); };
  // enqueue iteration j (jp == nullptr) or the iteration *jp (graph capture)
  auto iteration = [&](int64_t j, const int64_t* jp, hipStream_t q) {
    const int64_t jg = jp ? mres - 1 : j;  // grids cover the longest column
    if (jp) {
      if constexpr (std::is_same<TB, TW>::value) {
        using D = typename std::conditional<std::is_same<TB, double2>::value, GemmDesc, GemmDescX>::type;
        hipLaunchKernelGGL((point_matvec_kernel<D, TB>), dim3(1), dim3(64), 0, q, static_cast<D*>(dyn_desc), V,
                           vstride, jp);
      }
      dyn->launch(0, q);
    } else {
      mv.launch((size_t)j, q);  // w = A q_j
    }
    {
      // work: bytes of q_0..q_j and w for every right-hand side
      TimedLaunch tl(T_GMRES_DOTS, q, (vb * (double)(j + 1) + wb) * (double)nrhs * (double)n);
      if (n >= 2048 && nrhs < 16)
        hipLaunchKernelGGL((dots2_kernel<TB, TW, true>), dim3((unsigned)((jg + 4) / 4 * nrhs)), dim3(256), 0, q, V,
                           vstride, w, n, nrhs, j, gs, jp);
      else
        hipLaunchKernelGGL((dots2_kernel<TB, TW, false>), dim3((unsigned)((jg + 4) / 4 * nrhs)), dim3(256), 0, q, V,
                           vstride, w, n, nrhs, j, gs, jp);
    }
    hipLaunchKernelGGL(column_kernel, dim3((unsigned)nrhs), dim3(256), 0, q, gs, mres, j, nrhs, 1, jp);
    {
      // work: bytes of q_0..q_{j-1} read, q_j and w read and written, and
      // the j + j (j + 1) / 2 entries of H read for p = H a
      const double hr = (double)j + 0.5 * (double)j * (double)(j + 1);
      TimedLaunch tl(T_GMRES_UPDATE, q, ((vb * (double)(j + 2) + 2.0 * wb) * (double)n + 16.0 * hr) * (double)nrhs);
      const int64_t nhb = (jg + 1) * ng;
      if (gs.split > 1) {
        hipLaunchKernelGGL((dcgs_update_kernel<TB, TW, true>), dim3((unsigned)(nhb + (int64_t)np * nrhs * gs.split)),
                           dim3(512), 0, q, V, vstride, w, n, nrhs, mres, j, np, gs, part, jp);
        hipLaunchKernelGGL((dcgs_finish_kernel<TB, TW>), dim3((unsigned)((int64_t)np * nrhs)), dim3(64), 0, q, V,
                           vstride, w, n, nrhs, j, np, gs, part, jp);
      } else {
        hipLaunchKernelGGL((dcgs_update_kernel<TB, TW, false>), dim3((unsigned)(nhb + (int64_t)np * nrhs)), dim3(512),
                           0, q, V, vstride, w, n, nrhs, mres, j, np, gs, part, jp);
      }
    }
    hipLaunchKernelGGL((normalize_kernel<TB, TW>), grid2(n, nrhs), dim3(256), 0, q, w, V, vstride, n, part, np, gs,
                       mres, j, nrhs, jp, qd);
    if (jp) hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, q, jdev, (int64_t)1, 1);
    CBFM_HIP(hipGetLastError());
  };
  int pending = 0;  // flag copies queued in this cycle
  int64_t j = 0;
  bool done = false;
  auto check = [&]() {
    if (pending > 0 && all_done(flags.wait())) return true;
    flags.post(gs.active, s);
    ++pending;
    return false;
  };
  if (dyn && mres >= check_every && max_iter - total >= check_every) {
    hipStream_t cs;
    CBFM_HIP(hipStreamCreate(&cs));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        for (int q = 0; q < check_every; ++q) iteration(0, jdev, cs);
      } catch (...) {
        (void)hipStreamEndCapture(cs, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamSynchronize(cs);
        scratch_forget_stream(cs);
        (void)hipStreamDestroy(cs);
        throw;
      }
      e = hipStreamEndCapture(cs, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamSynchronize(cs);
    scratch_forget_stream(cs);
    (void)hipStreamDestroy(cs);
    CBFM_HIP(e);
    hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, jdev, (int64_t)0, 0);
    try {
      while (j + check_every <= mres && total + check_every <= max_iter) {
        CBFM_HIP(hipGraphLaunch(exec, s));
        j += check_every;
        total += check_every;
        if (check()) {
          done = true;
          break;
        }
      }
    } catch (...) {
      (void)hipGraphExecDestroy(exec);
      throw;
    }
    CBFM_HIP(hipGraphExecDestroy(exec));
  }
  for (; !done && j < mres && total < max_iter; ++j) {
    iteration(j, nullptr, s);
    ++total;
    if ((j + 1) % check_every == 0 && check()) {
      ++j;
      break;
    }
  }
  // the last column of the cycle, taken without the delayed correction
  if (j > 0) hipLaunchKernelGGL(column_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, gs, mres, j, nrhs, 0, nullptr);
  hipLaunchKernelGGL(backsolve_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, gs, mres, nrhs);
  // x += Q y, or Z y for flexible GMRES (the preconditioned vectors z_j)
  hipLaunchKernelGGL(x_update_kernel<TB>, dim3((unsigned)((int64_t)np * nrhs)), dim3(512), 0, s, gs, xb ? xb : V,
                     vstride, x, n, nrhs,
                     np);
  CBFM_HIP(hipGetLastError());
}

// ------------------------------------------------------------- s-step cycles
// Communication-avoiding form of the same GMRES (double arithmetic, dense
// double operator): per block of S iterations from the newest basis vector
// q_j, the Newton basis z_i = (A - theta_i) z_{i-1} / sigma_i (z_0 = q_j,
// i = 1..S) is formed by S matrix-vector products, orthogonalised against
// q_0..q_j by two block Gram-Schmidt passes (C = Q^H Z, Z -= Q C, twice)
// and within itself by two Cholesky QR passes (Z = U R), so that the basis
// is read four times per S iterations instead of twice per iteration.  With
// t_i the coordinates of z_i in [Q, U] (t_0 = e_j, t_i = [C_i; R_i]) and
// A z_{i-1} = sigma_i z_i + theta_i z_{i-1}, the new Hessenberg columns
// j..j+S-1 are (T_next - [H_old T_old; 0]) T_new^{-1}, where T_next holds
// sigma_i t_i + theta_i t_{i-1}, T_old the rows of t_0..t_{S-1} below j and
// T_new their rows j..j+S-1 (upper triangular).  The shifts are the Ritz
// values of a first plain cycle of S iterations in Leja order.

// z = u - theta q (written to basis slot jd, q = slot jd - 1) and the
// partial sums of |z|^2 of each 256-row block
__global__ void __launch_bounds__(256) newton_kernel(const double2* __restrict__ u, double2* __restrict__ V,
                                                     int64_t vstride, int64_t n, int64_t jd,
                                                     const double2* __restrict__ theta, int S, int ti,
                                                     GmresState st, double* __restrict__ part) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (!st.active[c]) return;  // uniform over the block
  double q2 = 0;
  if (k < n) {
    const double2 th = theta[c * S + ti];
    const double2 q = V[(jd - 1) * vstride + c * n + k], w = u[c * n + k];
    const double2 z = make_double2(w.x - (th.x * q.x - th.y * q.y), w.y - (th.x * q.y + th.y * q.x));
    V[jd * vstride + c * n + k] = z;
    q2 = z.x * z.x + z.y * z.y;
  }
  __shared__ double sh[4];
  q2 = wave_sum(q2);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q2;
  __syncthreads();
  if (threadIdx.x == 0) part[c * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// sigma = sqrt(sum of the partial sums); slot jd /= sigma
__global__ void __launch_bounds__(256) nscale_kernel(double2* __restrict__ V, int64_t vstride, int64_t n, int64_t jd,
                                                     const double* __restrict__ part, int np, double* __restrict__ sig,
                                                     int S, int ti, GmresState st) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (!st.active[c]) return;
  double q = 0;
  for (int b = 0; b < np; ++b) q += part[c * np + b];
  const double sg = sqrt(q);
  if (blockIdx.x == 0 && threadIdx.x == 0) sig[c * S + ti] = sg;
  if (k < n) {
    const double r = sg > 0 ? 1.0 / sg : 0.0;
    double2* p = V + jd * vstride + c * n + k;
    *p = make_double2(p->x * r, p->y * r);
  }
}

// out[c][l][i] = sum_k conj(L_l[k]) R_i[k] for l < nv, i < S: left vector l
// of right-hand side c at L + l ls + c lc, right vector i at R + i rs + c rc.
// One block of four wavefronts per right-hand side and run of four left
// vectors; the threads take every 256th row with the S right values of the
// row loaded once for the four left vectors, and the wavefronts are summed
// through LDS in a fixed order.  (GRAM: the same for a block's own Gram
// matrix, a launch of its own name for the profiles.)
template <int S, bool GRAM>
__global__ void __launch_bounds__(256) block_dots_kernel(const double2* __restrict__ L, int64_t ls, int64_t lc,
                                                         const double2* __restrict__ R, int64_t rs, int64_t rc,
                                                         int64_t n, int64_t nv, double2* __restrict__ out, int64_t ost,
                                                         GmresState st) {
  const int64_t runs = (nv + 3) / 4;
  const int64_t run = blockIdx.x % runs, c = blockIdx.x / runs;
  if (!st.active[c]) return;  // uniform over the block
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t l0 = run * 4;
  const int cnt = (int)std::min<int64_t>(4, nv - l0);
  const double2* Lc = L + l0 * ls + c * lc;
  const double2* Rc = R + c * rc;
  double2 acc[4][S];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < S; ++i) acc[t][i] = make_double2(0, 0);
  for (int64_t k = threadIdx.x; k < n; k += 256) {
    double2 v[4], z[S];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = Lc[(t < cnt ? t : 0) * ls + k];  // vectors past nv: discarded
#pragma unroll
    for (int i = 0; i < S; ++i) z[i] = Rc[i * rs + k];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < S; ++i) acc[t][i] = cadd(acc[t][i], cconjmul(v[t], z[i]));
  }
  __shared__ double2 sh[4][4][S];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const double re = wave_sum(acc[t][i].x), im = wave_sum(acc[t][i].y);
      if (lane == 0) sh[wv][t][i] = make_double2(re, im);
    }
  __syncthreads();
  const int e = threadIdx.x;
  if (e < 4 * S && e / S < cnt) {
    const int t = e / S, i = e % S;
    const double2 a = cadd(cadd(sh[0][t][i], sh[1][t][i]), cadd(sh[2][t][i], sh[3][t][i]));
    out[c * ost + (l0 + t) * S + i] = a;
  }
}

// Z_i[k] -= sum_{l < nv} C[c][l][i] Q_l[k] (Q_l = V + l vstride + c n, Z_i in
// the basis slots after q_j): eight wavefronts take 128 consecutive rows of
// one right-hand side (two per lane), wavefront v summing over l = v mod 8;
// the partial sums are added through LDS in wavefront order.
template <int S>
__global__ void __launch_bounds__(512) block_update_kernel(const double2* __restrict__ V, int64_t vstride,
                                                           double2* __restrict__ Z, int64_t n, int64_t nv,
                                                           const double2* __restrict__ C, int64_t cst, int np,
                                                           GmresState st) {
  constexpr int RPL = 2;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t c = blockIdx.x / np, rb = blockIdx.x % np;
  if (!st.active[c]) return;  // uniform over the block
  int64_t kk[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int64_t k = (rb * RPL + r) * 64 + lane;
    kk[r] = k < n ? k : 0;  // rows past n: a valid row, discarded
  }
  const double2* Q = V + c * n;
  const double2* Cc = C + c * cst * S;
  double2 acc[RPL][S];
#pragma unroll
  for (int r = 0; r < RPL; ++r)
#pragma unroll
    for (int i = 0; i < S; ++i) acc[r][i] = make_double2(0, 0);
  int64_t l = wv;
  for (; l + 8 < nv; l += 16) {  // two left vectors at a time, their loads issued together
    double2 q0[RPL], q1[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      q0[r] = Q[l * vstride + kk[r]];
      q1[r] = Q[(l + 8) * vstride + kk[r]];
    }
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const double2 a0 = Cc[l * S + i], a1 = Cc[(l + 8) * S + i];
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[r][i] = cadd(acc[r][i], cadd(cmul(a0, q0[r]), cmul(a1, q1[r])));
    }
  }
  for (; l < nv; l += 8) {
    double2 q0[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) q0[r] = Q[l * vstride + kk[r]];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const double2 a0 = Cc[l * S + i];
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[r][i] = cadd(acc[r][i], cmul(a0, q0[r]));
    }
  }
  __shared__ double2 sh[RPL][64][S];
  for (int w = 0; w < 8; ++w) {
    if (wv == w) {
#pragma unroll
      for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int i = 0; i < S; ++i) sh[r][lane][i] = w == 0 ? acc[r][i] : cadd(sh[r][lane][i], acc[r][i]);
    }
    __syncthreads();
  }
  if (wv != 0) return;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int64_t k = (rb * RPL + r) * 64 + lane;
    if (k >= n) continue;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      double2* p = Z + i * vstride + c * n + k;
      const double2 a = sh[r][lane][i];
      *p = make_double2(p->x - a.x, p->y - a.y);
    }
  }
}

// Cholesky factor of one right-hand side's Gram matrix G = R^H R (R upper,
// S x S), its inverse, and Rt = R (first pass) or R Rt; a pivot not above
// 1e-28 of G's largest diagonal entry marks a breakdown (broken[c] = 1).
// G is staged in LDS, one thread factors and inverts it there, and the
// results are written by S x S threads.
template <int S>
__global__ void __launch_bounds__(64) chol_kernel(const double2* __restrict__ G, double2* __restrict__ Rinv,
                                                  double2* __restrict__ Rt, int first, GmresState st,
                                                  int32_t* __restrict__ broken) {
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  if (!st.active[c]) return;  // uniform over the block
  __shared__ double2 Gs[S][S], R[S][S], Ri[S][S];
  __shared__ int bad;
  for (int e = tid; e < S * S; e += 64) Gs[e / S][e % S] = G[c * S * S + e];
  __syncthreads();
  if (tid == 0) {
    double gmax = 0;
    for (int i = 0; i < S; ++i) gmax = fmax(gmax, Gs[i][i].x);
    int b = !(gmax > 0);
    for (int i = 0; i < S && !b; ++i) {
      double d = Gs[i][i].x;
      for (int p = 0; p < i; ++p) d -= R[p][i].x * R[p][i].x + R[p][i].y * R[p][i].y;
      if (!(d > 1e-28 * gmax)) {
        b = 1;
        break;
      }
      const double rii = sqrt(d);
      R[i][i] = make_double2(rii, 0);
      for (int q = i + 1; q < S; ++q) {
        double2 a = Gs[i][q];
        for (int p = 0; p < i; ++p) a = make_double2(a.x - (R[p][i].x * R[p][q].x + R[p][i].y * R[p][q].y),
                                                     a.y - (R[p][i].x * R[p][q].y - R[p][i].y * R[p][q].x));
        R[i][q] = make_double2(a.x / rii, a.y / rii);
      }
      for (int q = 0; q < i; ++q) R[i][q] = make_double2(0, 0);
    }
    if (!b) {
      for (int i = S - 1; i >= 0; --i) {
        Ri[i][i] = make_double2(1.0 / R[i][i].x, 0);
        for (int q = i + 1; q < S; ++q) {
          double2 a = make_double2(0, 0);
          for (int p = i; p < q; ++p) a = cadd(a, cmul(Ri[i][p], R[p][q]));
          Ri[i][q] = make_double2(-a.x / R[q][q].x, -a.y / R[q][q].x);
        }
        for (int q = 0; q < i; ++q) Ri[i][q] = make_double2(0, 0);
      }
    }
    bad = b;
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) broken[c] = 1;
    return;
  }
  double2* Ric = Rinv + c * S * S;
  double2* Rtc = Rt + c * S * S;
  double2 nt[(S * S + 63) / 64];
#pragma unroll
  for (int u = 0; u < (S * S + 63) / 64; ++u) {
    const int e = tid + 64 * u;
    if (e >= S * S) break;
    const int i = e / S, q = e % S;
    Ric[e] = Ri[i][q];
    if (first) {
      nt[u] = R[i][q];
    } else {
      double2 a = make_double2(0, 0);
      for (int p = i; p <= q; ++p) a = cadd(a, cmul(R[i][p], Rtc[p * S + q]));
      nt[u] = a;
    }
  }
  __syncthreads();  // every old Rt entry read before any is replaced
#pragma unroll
  for (int u = 0; u < (S * S + 63) / 64; ++u) {
    const int e = tid + 64 * u;
    if (e < S * S) Rtc[e] = nt[u];
  }
}

// Z <- Z R^{-1} in place (Z_i = the basis slot after q_j plus i): each
// thread takes one row of every right-hand side's S vectors.
template <int S>
__global__ void __launch_bounds__(256) trmul_kernel(double2* __restrict__ Z, int64_t vstride, int64_t n,
                                                    const double2* __restrict__ Rinv, GmresState st) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (!st.active[c]) return;  // uniform over the block
  __shared__ double2 Ri[S][S];
  if (threadIdx.x < S * S) Ri[threadIdx.x / S][threadIdx.x % S] = Rinv[c * S * S + threadIdx.x];
  __syncthreads();
  if (k >= n) return;
  double2 z[S];
#pragma unroll
  for (int i = 0; i < S; ++i) z[i] = Z[i * vstride + c * n + k];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    double2 a = make_double2(0, 0);
#pragma unroll
    for (int p = 0; p <= i; ++p) a = cadd(a, cmul(z[p], Ri[p][i]));
    Z[i * vstride + c * n + k] = a;
  }
}

// C1 += C2 over rows 0..j of every right-hand side (the two Gram-Schmidt
// passes' coefficients, summed once per block of iterations)
__global__ void csum_kernel(double2* __restrict__ C1, const double2* __restrict__ C2, int64_t cst, int S, int64_t j,
                            GmresState st) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (!st.active[c] || e >= (j + 1) * S) return;
  C1[c * cst * S + e] = cadd(C1[c * cst * S + e], C2[c * cst * S + e]);
}

// T_new^{-1} of one right-hand side into LDS (thread 0): T_new's column 0
// is e_0 and its column q >= 1 is [C[j][q-1]; R[0..q-1][q-1]].
template <int S>
__device__ void tnew_inverse(const double2 (&Rs)[S][S], const double2 (&cj)[S], double2 (&Tinv)[S][S]) {
  double2 Tn[S][S];
  for (int r = 0; r < S; ++r)
    for (int q = 0; q < S; ++q)
      Tn[r][q] = q == 0 ? make_double2(r == 0 ? 1.0 : 0.0, 0.0)
                        : (r == 0 ? cj[q - 1] : (r - 1 <= q - 1 ? Rs[r - 1][q - 1] : make_double2(0, 0)));
  for (int i = S - 1; i >= 0; --i) {
    const double2 d = Tn[i][i];
    const double dd = d.x * d.x + d.y * d.y;
    Tinv[i][i] = make_double2(d.x / dd, -d.y / dd);
    for (int q = i + 1; q < S; ++q) {
      double2 a = make_double2(0, 0);
      for (int p = i; p < q; ++p) a = cadd(a, cmul(Tinv[i][p], Tn[p][q]));
      const double2 e = Tn[q][q];
      const double ee = e.x * e.x + e.y * e.y;
      const double2 v = cmul(a, make_double2(e.x / ee, -e.y / ee));
      Tinv[i][q] = make_double2(-v.x, -v.y);
    }
    for (int q = 0; q < i; ++q) Tinv[i][q] = make_double2(0, 0);
  }
}

// Rows r0..r0+63 of the Hessenberg columns j..j+S-1 of one right-hand side,
// stored un-rotated in H (column-major, M1 rows per column):
// (T_next - [H_old T_old; 0]) T_new^{-1}.  Four wavefronts split the sum
// over l of H_old T_old (l = w mod 4), a lane per row, and wavefront 0
// adds their parts and forms the rows.  C holds C1 + C2 (csum_kernel).
template <int S>
__global__ void __launch_bounds__(256) sstep_hcols_kernel(GmresState st, double2* __restrict__ H, int64_t M1,
                                                          int64_t HS, const double2* __restrict__ C, int64_t cst,
                                                          const double2* __restrict__ Rt,
                                                          const double* __restrict__ sig,
                                                          const double2* __restrict__ theta,
                                                          const int32_t* __restrict__ broken, int64_t j) {
  const int64_t c = blockIdx.y;
  if (!st.active[c] || broken[c]) return;  // uniform over the block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double2 Tinv[S][S], Rs[S][S], th[S], cj[S];
  __shared__ double sg[S];
  __shared__ double2 part[3][64][S];
  const double2* Cc = C + c * cst * S;
  if (tid < S * S) Rs[tid / S][tid % S] = Rt[c * S * S + tid];
  if (tid < S) {
    th[tid] = theta[c * S + tid];
    sg[tid] = sig[c * S + tid];
    cj[tid] = Cc[j * S + tid];
  }
  __syncthreads();
  if (tid == 0) tnew_inverse<S>(Rs, cj, Tinv);
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const int64_t rr = r <= j ? r : j;  // rows past j: a valid row of H_old, discarded
  double2* Hc = H + c * HS;
  double2 acc[S];
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = make_double2(0, 0);
  // H[r][l] = 0 for l < r - 1: the wavefronts start at the block's first such l
  const int64_t lstart = blockIdx.x * 64 > 0 ? blockIdx.x * 64 - 1 : 0;
#pragma unroll 4
  for (int64_t l = lstart + wv; l < j; l += 4) {
    const double2 hv = Hc[l * M1 + rr];
    const double2 h = l + 1 >= r ? hv : make_double2(0, 0);
#pragma unroll
    for (int q = 1; q < S; ++q) acc[q] = cadd(acc[q], cmul(h, Cc[l * S + q - 1]));
  }
  if (wv > 0) {
#pragma unroll
    for (int q = 0; q < S; ++q) part[wv - 1][lane][q] = acc[q];
  }
  __syncthreads();
  if (wv > 0 || r > j + S) return;
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = cadd(acc[q], cadd(cadd(part[0][lane][q], part[1][lane][q]), part[2][lane][q]));
  // t_i[r]: t_0 = e_j; t_i = [C_{i-1}; R_{i-1}]
  auto tval = [&](int i) -> double2 {
    if (i == 0) return make_double2(r == j ? 1.0 : 0.0, 0.0);
    if (r <= j) return Cc[r * S + i - 1];
    const int64_t k = r - j - 1;
    return k <= i - 1 ? Rs[k][i - 1] : make_double2(0, 0);
  };
  double2 X[S];
  double2 tprev = tval(0);
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const double2 tn = tval(q + 1);
    X[q] = cadd(make_double2(sg[q] * tn.x, sg[q] * tn.y), cmul(th[q], tprev));
    if (r <= j && q >= 1) X[q] = make_double2(X[q].x - acc[q].x, X[q].y - acc[q].y);
    tprev = tn;
  }
#pragma unroll
  for (int q = 0; q < S; ++q) {
    double2 a = make_double2(0, 0);
#pragma unroll
    for (int p = 0; p <= q; ++p) a = cadd(a, cmul(X[p], Tinv[p][q]));
    Hc[(j + q) * M1 + r] = r <= j + q + 1 ? a : make_double2(0, 0);
  }
}

// The new Hessenberg columns j..j+S-1 of one right-hand side rotated into
// R.  The earlier rotations act on each new column as an affine recurrence
// in the carried entry (a -> -conj(s_l) a + conj(c_l) H[l+1]), so T = 256/S
// threads per column each compose the maps of a run of rotations, a scan
// over the runs (in LDS) gives each run its incoming entry, and the runs are
// replayed in parallel.  Thread 0 then applies this block's rotations in
// order, forms each new rotation, and updates g, the residual estimate and
// the stop test as column_kernel does.  A right-hand side whose Cholesky QR
// broke down keeps the columns before this block and ends its cycle.
template <int S>
__global__ void __launch_bounds__(256) sstep_givens_kernel(GmresState st, const double2* __restrict__ H, int64_t M1,
                                                           int64_t HS, const int32_t* __restrict__ broken, int64_t j,
                                                           int64_t m, int64_t nrhs) {
  constexpr int T = 256 / S;  // threads per column
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  if (!st.active[c]) return;  // uniform over the block
  if (broken[c]) {
    if (tid == 0) st.active[c] = 0;
    return;
  }
  __shared__ double2 pc[S];
  __shared__ double2 mapa[S][T], mapb[S][T], inc[S][T];
  const double2* Hc = H + c * HS;
  double2* Rc = st.R + c * (m + 1) * m;
  double2* cs = st.cs + c * m;
  double2* sn = st.sn + c * m;
  const int q = tid / T, t = tid % T;
  const int64_t k = j + q;
  const int64_t per = (j + T - 1) / T, l0 = std::min<int64_t>(j, t * per), l1 = std::min<int64_t>(j, l0 + per);
  // the run's composed map a -> A a + B
  double2 A = make_double2(1, 0), B = make_double2(0, 0);
  for (int64_t l = l0; l < l1; ++l) {
    const double2 cl = cs[l], sl = sn[l], b = Hc[k * M1 + l + 1];
    const double2 al = make_double2(-sl.x, sl.y), bl = cmul(make_double2(cl.x, -cl.y), b);
    A = cmul(al, A);
    B = cadd(cmul(al, B), bl);
  }
  mapa[q][t] = A;
  mapb[q][t] = B;
  __syncthreads();
  if (t == 0) {  // incoming entry of every run of this column, in run order
    double2 a = Hc[k * M1];
    for (int u = 0; u < T; ++u) {
      inc[q][u] = a;
      a = cadd(cmul(mapa[q][u], a), mapb[q][u]);
    }
    pc[q] = a;
  }
  __syncthreads();
  {
    double2 a = inc[q][t];
    for (int64_t l = l0; l < l1; ++l) {
      const double2 cl = cs[l], sl = sn[l], b = Hc[k * M1 + l + 1];
      Rc[k * (m + 1) + l] = cadd(cmul(cl, a), cmul(sl, b));
      a = cadd(cmul(make_double2(-sl.x, sl.y), a), cmul(make_double2(cl.x, -cl.y), b));
    }
  }
  __syncthreads();
  if (tid != 0) return;
  const double bnorm = st.bnorm[c], tgt = st.tgt[c];
  for (int q = 0; q < S; ++q) {
    const int64_t k = j + q;
    double2 a = pc[q];
    for (int64_t l = j; l < k; ++l) {
      const double2 b = Hc[k * M1 + l + 1], cl = cs[l], sl = sn[l];
      Rc[k * (m + 1) + l] = cadd(cmul(cl, a), cmul(sl, b));
      a = cadd(cmul(make_double2(-sl.x, sl.y), a), cmul(make_double2(cl.x, -cl.y), b));
    }
    const double2 h = Hc[k * M1 + k + 1];
    const double den = sqrt(a.x * a.x + a.y * a.y + h.x * h.x + h.y * h.y);
    double2 cc = make_double2(1, 0), ss = make_double2(0, 0);
    if (den > 0) {
      cc = make_double2(a.x / den, -a.y / den);  // conj(a)/den
      ss = make_double2(h.x / den, -h.y / den);  // conj(h)/den
    }
    cs[k] = cc;
    sn[k] = ss;
    Rc[k * (m + 1) + k] = make_double2(den, 0);
    const double2 gj = st.g[k * nrhs + c];
    const double2 gn = make_double2(-(ss.x * gj.x + ss.y * gj.y), -(ss.x * gj.y - ss.y * gj.x));
    st.g[(k + 1) * nrhs + c] = gn;
    st.g[k * nrhs + c] = cmul(cc, gj);
    const double ra = sqrt(gn.x * gn.x + gn.y * gn.y);
    st.res[c] = ra / bnorm;
    st.kc[c] = (int32_t)(k + 1);
    st.its[c] += 1;
    if (ra <= tgt || den == 0.0 || k + 1 >= m) {
      st.active[c] = 0;
      return;
    }
  }
}

// Eigenvalues of an n x n upper Hessenberg matrix (row-major): shifted QR
// steps with Givens rotations on the active window, Wilkinson shifts (an
// exceptional shift every 11 steps), deflation at negligible subdiagonal
// entries; after 300 steps on one window its diagonal is taken as it is.
static std::vector<std::complex<double>> hessenberg_eigenvalues(std::vector<std::complex<double>> H, int n) {
  typedef std::complex<double> cx;
  std::vector<cx> ev;
  int hi = n - 1, steps = 0;
  while (hi >= 0) {
    if (hi == 0) {
      ev.push_back(H[0]);
      break;
    }
    int lo = hi;
    while (lo > 0 && std::abs(H[lo * n + lo - 1]) > 1e-14 * (std::abs(H[lo * n + lo]) + std::abs(H[(lo - 1) * n + lo - 1])))
      --lo;
    if (lo == hi) {
      ev.push_back(H[hi * n + hi]);
      --hi;
      steps = 0;
      continue;
    }
    if (++steps > 300) {
      for (int k = lo; k <= hi; ++k) ev.push_back(H[k * n + k]);
      hi = lo - 1;
      steps = 0;
      continue;
    }
    const cx a = H[(hi - 1) * n + hi - 1], b = H[(hi - 1) * n + hi], c = H[hi * n + hi - 1], d = H[hi * n + hi];
    const cx half_tr = 0.5 * (a + d), disc = std::sqrt(half_tr * half_tr - (a * d - b * c));
    cx mu = std::abs(half_tr + disc - d) < std::abs(half_tr - disc - d) ? half_tr + disc : half_tr - disc;
    if (steps % 11 == 0) mu += std::abs(c);
    for (int k = lo; k <= hi; ++k) H[k * n + k] -= mu;
    std::vector<double> rc(n);
    std::vector<cx> rs(n);
    for (int k = lo; k < hi; ++k) {  // H <- G_k H (rows k, k+1)
      const cx x = H[k * n + k], y = H[(k + 1) * n + k];
      const double r = std::hypot(std::abs(x), std::abs(y));
      double cc = 1;
      cx ss = 0;
      if (r > 0) {
        cc = std::abs(x) / r;
        ss = (std::abs(x) > 0 ? x / std::abs(x) : cx(1, 0)) * std::conj(y) / r;
      }
      rc[k] = cc;
      rs[k] = ss;
      for (int q = k; q <= hi; ++q) {
        const cx u = H[k * n + q], v = H[(k + 1) * n + q];
        H[k * n + q] = cc * u + ss * v;
        H[(k + 1) * n + q] = -std::conj(ss) * u + cc * v;
      }
    }
    for (int k = lo; k < hi; ++k) {  // H <- H G_k^H (columns k, k+1)
      const double cc = rc[k];
      const cx ss = rs[k];
      for (int r = lo; r <= std::min(k + 2, hi); ++r) {
        const cx u = H[r * n + k], v = H[r * n + k + 1];
        H[r * n + k] = cc * u + std::conj(ss) * v;
        H[r * n + k + 1] = -ss * u + cc * v;
      }
    }
    for (int k = lo; k <= hi; ++k) H[k * n + k] += mu;
  }
  return ev;
}

// Leja order: the value of largest modulus first, then each time the one
// farthest (by product of distances) from those already taken.
static std::vector<std::complex<double>> leja_order(std::vector<std::complex<double>> v) {
  std::vector<std::complex<double>> out;
  while (!v.empty()) {
    size_t best = 0;
    double bv = -1;
    for (size_t i = 0; i < v.size(); ++i) {
      double p = out.empty() ? std::abs(v[i]) : 1.0;
      for (const auto& o : out) p *= std::abs(v[i] - o);
      if (p > bv) {
        bv = p;
        best = i;
      }
    }
    out.push_back(v[best]);
    v.erase(v.begin() + (int64_t)best);
  }
  return out;
}

// The device buffers of s-step cycles of length m (a multiple of S).
struct SStep {
  int S;
  int64_t n, nrhs, m, M1, HS, cst;
  Scratch C1, C2, G, Rinv, Rt, sig, theta, broken;
  // the dot passes C = Q^H Z as products of the row-block GEMM, one per
  // right-hand side: descriptor 2 b + pass for block b (on the host and
  // the device) and the workspace of their K-split parts
  std::vector<GemmDesc> dots;
  std::unique_ptr<Scratch> dots_dev, dots_ws;
  SStep(int S_, int64_t n_, int64_t nrhs_, int64_t m_, hipStream_t s)
      : S(S_), n(n_), nrhs(nrhs_), m(m_), M1(m_ + S_ + 1), HS((m_ + S_) * (m_ + S_ + 1)), cst(m_ + 1),
        C1(nrhs_ * (m_ + 1) * S_ * sizeof(double2), s), C2(nrhs_ * (m_ + 1) * S_ * sizeof(double2), s),
        G(nrhs_ * S_ * S_ * sizeof(double2), s), Rinv(nrhs_ * S_ * S_ * sizeof(double2), s),
        Rt(nrhs_ * S_ * S_ * sizeof(double2), s), sig(nrhs_ * S_ * sizeof(double), s),
        theta(nrhs_ * S_ * sizeof(double2), s), broken(nrhs_ * sizeof(int32_t), s) {}
  // block b (j = b S) of pass p: C_p[c][l][i] = sum_k conj(q_l[k]) z_i[k]
  // for l <= j, i < S, right-hand side c (q_l = V + l vstride + c n, the
  // block's z_i in the basis slots after q_j)
  void prepare_dots(const double2* V, int64_t vstride, hipStream_t s) {
    const int64_t nb = m / S;
    dots.clear();
    size_t ws = 0;
    for (int64_t b = 0; b < nb; ++b)
      for (int p = 0; p < 2; ++p) {
        const int64_t j = b * S;
        GemmDesc d = gemm(V, vstride, OP_R, V + (j + 1) * vstride, vstride, OP_T,
                          (p == 0 ? C1 : C2).as<double2>(), S, j + 1, S, n);
        dots.push_back(d);
        ws = std::max(ws, panel_batch_ws_bytes(d, nrhs));
      }
    dots_dev.reset(new Scratch(std::max<size_t>(1, dots.size()) * sizeof(GemmDesc), s));
    if (!dots.empty()) {
      CBFM_HIP(hipMemcpyAsync(dots_dev->p, dots.data(), dots.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
      CBFM_HIP(hipStreamSynchronize(s));  // `dots` may be rebuilt while the copy is in flight otherwise
    }
    dots_ws.reset(new Scratch(ws, s));
  }
};

// Shifts of every right-hand side from the Hessenberg matrix of a plain
// cycle of length m1 (> S): the Ritz values of its leading S x S block (of
// its first its[c] columns when fewer), in Leja order, zeros when none.
static void sstep_shifts(SStep& ss, const GmresState& gs, int64_t m1, const std::vector<int32_t>& its, hipStream_t s) {
  const int S = ss.S;
  const int64_t nrhs = ss.nrhs;
  std::vector<double2> Hh((size_t)(m1 + 1) * m1 * nrhs);
  CBFM_HIP(hipMemcpyAsync(Hh.data(), gs.H, Hh.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  CBFM_HIP(hipStreamSynchronize(s));
  std::vector<double2> th((size_t)nrhs * S, make_double2(0, 0));
  for (int64_t c = 0; c < nrhs; ++c) {
    const int k = (int)std::min<int64_t>(S, its[c]);
    if (k < 1) continue;
    std::vector<std::complex<double>> Hk((size_t)k * k);
    for (int l = 0; l < k; ++l)
      for (int i = 0; i < k; ++i) {
        const double2 v = Hh[((size_t)l * m1 + i) * nrhs + c];
        Hk[(size_t)l * k + i] = (l <= i + 1 && std::isfinite(v.x) && std::isfinite(v.y)) ? std::complex<double>(v.x, v.y)
                                                                                        : std::complex<double>(0, 0);
      }
    const auto ev = leja_order(hessenberg_eigenvalues(Hk, k));
    for (int i = 0; i < S; ++i) {
      const auto z = ev[(size_t)i % ev.size()];
      th[(size_t)c * S + i] = make_double2(z.real(), z.imag());
    }
  }
  CBFM_HIP(hipMemcpyAsync(ss.theta.p, th.data(), th.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  CBFM_HIP(hipStreamSynchronize(s));  // th is host memory of this frame
}

// One s-step cycle of length ss.m from the normalised residual in V[0]
// (cycle_init done): blocks of S iterations, then the triangular solve and
// x += Q y.  Returns whether some right-hand side broke down (its cycle
// then ends at the last complete block).
static bool run_sstep_cycle(SStep& ss, const GemmPlan& matvec, double2* V, double2* u, int64_t vstride,
                            int64_t max_iter, int64_t& total, GmresState gs, double* part, int np, PinnedFlags& flags,
                            double2* x, double2* H, hipStream_t s) {
  const int S = ss.S;
  const int64_t n = ss.n, nrhs = ss.nrhs, m = ss.m;
  const int np256 = (int)((n + 255) / 256);
  CBFM_HIP(hipMemsetAsync(ss.broken.p, 0, nrhs * sizeof(int32_t), s));
  auto all_done = [&](const int32_t* a) { return std::none_of(a, a + nrhs, [](int32_t v) { return v != 0; }); };
  int pending = 0;
  for (int64_t b = 0; b * S < m && total + S <= max_iter; ++b) {
    const int64_t j = b * S;
    for (int i = 1; i <= S; ++i) {  // z_i = (A - theta_i) z_{i-1} / sigma_i into slot j + i
      matvec.launch((size_t)(j + i - 1), s);
      hipLaunchKernelGGL(newton_kernel, dim3((unsigned)np256, (unsigned)nrhs), dim3(256), 0, s, u, V, vstride, n, j + i,
                         ss.theta.as<double2>(), S, i - 1, gs, part);
      hipLaunchKernelGGL(nscale_kernel, dim3((unsigned)np256, (unsigned)nrhs), dim3(256), 0, s, V, vstride, n, j + i,
                         part, np256, ss.sig.as<double>(), S, i - 1, gs);
    }
    // two block Gram-Schmidt passes against q_0..q_j, then Cholesky QR twice
    double2* Z = V + (j + 1) * vstride;
    const int npu = (int)((n + 127) / 128);
    const double vb = 16.0 * (double)(j + 1) * (double)nrhs * (double)n;  // bytes of q_0..q_j
    for (int pass = 0; pass < 2; ++pass) {
      double2* Cp = pass == 0 ? ss.C1.as<double2>() : ss.C2.as<double2>();
      {
        TimedLaunch tl(T_GMRES_DOTS, s, vb + 16.0 * S * (double)nrhs * (double)n);
        const size_t di = (size_t)(2 * b + pass);
        panel_batch(ss.dots_dev->as<GemmDesc>() + di, ss.dots[di], nrhs, n, n, ss.cst * S, ss.dots_ws->as<double>(), s);
      }
      {
        TimedLaunch tl(T_GMRES_UPDATE, s, vb + 32.0 * S * (double)nrhs * (double)n);
        if (S == 4)
          hipLaunchKernelGGL(block_update_kernel<4>, dim3((unsigned)(npu * nrhs)), dim3(512), 0, s, V, vstride, Z, n,
                             j + 1, Cp, ss.cst, npu, gs);
        else
          hipLaunchKernelGGL(block_update_kernel<8>, dim3((unsigned)(npu * nrhs)), dim3(512), 0, s, V, vstride, Z, n,
                             j + 1, Cp, ss.cst, npu, gs);
      }
    }
    const unsigned gr = (unsigned)(((S + 3) / 4) * nrhs);
    const dim3 gz((unsigned)((n + 255) / 256), (unsigned)nrhs);
    for (int pass = 0; pass < 2; ++pass) {  // Cholesky QR, in place
      if (S == 4) {
        hipLaunchKernelGGL((block_dots_kernel<4, true>), dim3(gr), dim3(256), 0, s, Z, vstride, n, Z, vstride, n, n,
                           (int64_t)S, ss.G.as<double2>(), (int64_t)S * S, gs);
        hipLaunchKernelGGL(chol_kernel<4>, dim3((unsigned)nrhs), dim3(64), 0, s, ss.G.as<double2>(),
                           ss.Rinv.as<double2>(), ss.Rt.as<double2>(), pass == 0, gs, ss.broken.as<int32_t>());
        hipLaunchKernelGGL(trmul_kernel<4>, gz, dim3(256), 0, s, Z, vstride, n, ss.Rinv.as<double2>(), gs);
      } else {
        hipLaunchKernelGGL((block_dots_kernel<8, true>), dim3(gr), dim3(256), 0, s, Z, vstride, n, Z, vstride, n, n,
                           (int64_t)S, ss.G.as<double2>(), (int64_t)S * S, gs);
        hipLaunchKernelGGL(chol_kernel<8>, dim3((unsigned)nrhs), dim3(64), 0, s, ss.G.as<double2>(),
                           ss.Rinv.as<double2>(), ss.Rt.as<double2>(), pass == 0, gs, ss.broken.as<int32_t>());
        hipLaunchKernelGGL(trmul_kernel<8>, gz, dim3(256), 0, s, Z, vstride, n, ss.Rinv.as<double2>(), gs);
      }
    }
    const unsigned nrb = (unsigned)((j + S + 1 + 63) / 64);
    hipLaunchKernelGGL(csum_kernel, dim3((unsigned)(((j + 1) * S + 255) / 256), (unsigned)nrhs), dim3(256), 0, s,
                       ss.C1.as<double2>(), ss.C2.as<double2>(), ss.cst, S, j, gs);
    if (S == 4) {
      hipLaunchKernelGGL(sstep_hcols_kernel<4>, dim3(nrb, (unsigned)nrhs), dim3(256), 0, s, gs, H, ss.M1, ss.HS,
                         ss.C1.as<double2>(), ss.cst, ss.Rt.as<double2>(), ss.sig.as<double>(), ss.theta.as<double2>(),
                         ss.broken.as<int32_t>(), j);
      hipLaunchKernelGGL(sstep_givens_kernel<4>, dim3((unsigned)nrhs), dim3(256), 0, s, gs, H, ss.M1, ss.HS,
                         ss.broken.as<int32_t>(), j, m, nrhs);
    } else {
      hipLaunchKernelGGL(sstep_hcols_kernel<8>, dim3(nrb, (unsigned)nrhs), dim3(256), 0, s, gs, H, ss.M1, ss.HS,
                         ss.C1.as<double2>(), ss.cst, ss.Rt.as<double2>(), ss.sig.as<double>(), ss.theta.as<double2>(),
                         ss.broken.as<int32_t>(), j);
      hipLaunchKernelGGL(sstep_givens_kernel<8>, dim3((unsigned)nrhs), dim3(256), 0, s, gs, H, ss.M1, ss.HS,
                         ss.broken.as<int32_t>(), j, m, nrhs);
    }
    CBFM_HIP(hipGetLastError());
    total += S;
    if (pending > 0 && all_done(flags.wait())) break;
    flags.post(gs.active, s);
    ++pending;
  }
  hipLaunchKernelGGL(backsolve_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, gs, m, nrhs);
  hipLaunchKernelGGL(x_update_kernel<double2>, dim3((unsigned)((int64_t)np * nrhs)), dim3(512), 0, s, gs, V, vstride,
                     x, n, nrhs, np);
  CBFM_HIP(hipGetLastError());
  std::vector<int32_t> br(nrhs);
  CBFM_HIP(hipMemcpyAsync(br.data(), ss.broken.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CBFM_HIP(hipStreamSynchronize(s));
  return std::any_of(br.begin(), br.end(), [](int32_t v) { return v != 0; });
}

// r = A x in double for row-stored vectors x (nrhs x n), A float (lda):
// the matrix-core product with float operands, double accumulation output.
static void apply_op32(const float2* A, int64_t lda, int64_t n, int64_t nrhs, const double2* x, double2* r,
                       hipStream_t s) {
  std::vector<GemmDescX> d{gemmx(A, 0, lda, OP_N, x, 1, n, OP_T, r, 1, n, n, nrhs, n)};
  d[0].transC = 1;
  xgemm_batched(d, XG_FP32, s);
}

namespace {
// w = A q_j through a composite operator
struct OpMV {
  const KrylovOp* op;
  void launch(size_t j, hipStream_t q) const { op->launch((int64_t)j, q); }
};
}  // namespace

GmresResult gmres_run(KrylovOp& op, int64_t n, int64_t nrhs, const double2* b, double2* x, const GmresSpec& p,
                      hipStream_t s) {
  int64_t lda64 = 0, lda32 = 0;
  const double2* A64 = op.dense64(&lda64);
  const float2* A32in = op.dense32(&lda32);
  const bool dense = A64 != nullptr || A32in != nullptr;
  // a float-only operator runs float cycles (its residuals in float too)
  const bool f32 = p.f32 || (A32in != nullptr && A64 == nullptr);
  CBFM_REQUIRE(dense || !f32, CBFM_E_ARG, "float Krylov cycles need a dense operator");
  // compressed basis: double arithmetic, the basis stored in float
  const bool b32 = p.basis32 && !f32;
  CBFM_REQUIRE(!b32 || A64 != nullptr, CBFM_E_ARG, "a float-stored basis needs a dense double operator");
  const int S = p.sstep;
  CBFM_REQUIRE(S == 0 || ((S == 4 || S == 8) && A64 != nullptr && !f32 && !b32 && !p.graph && op.xbasis() == nullptr),
               CBFM_E_ARG, "s-step cycles take blocks of 4 or 8 with a dense double operator, a double basis, no graphs");
  CBFM_REQUIRE(p.tol > 0 && p.max_iter >= 1 && p.restart >= 1, CBFM_E_ARG, "bad solver parameters");
  if (p.block) {
    CBFM_REQUIRE(dense && !p.f32 && !b32 && S == 0 && !p.graph && op.xbasis() == nullptr, CBFM_E_ARG,
                 "block GMRES takes a dense operator, a double basis, no s-step cycles and no graphs");
    return block_gmres_run(A64, lda64, A64 ? nullptr : A32in, lda32, n, nrhs, b, x, p, s);
  }
  const int64_t mres = std::min<int64_t>(p.restart, std::max<int64_t>(p.max_iter, 1));
  // The plain form keeps the Krylov basis in double; the mixed form keeps it
  // and the operator in float and refines: every cycle starts from the
  // residual b - A x formed in double, and stops once it has reduced that
  // residual by inner_tol (or reached tol).  The compressed-basis form
  // keeps the plain form's arithmetic and stores only the basis in float
  // (half the bytes of the Arnoldi passes); its Arnoldi relation then holds
  // to float rounding, so its cycles stop and restart as the mixed form's.
  const double inner = f32 || b32 ? (p.inner_tol > 0 ? p.inner_tol : 1e-6) : 0.0;
  const size_t vsz = f32 || b32 ? sizeof(float2) : sizeof(double2);
  Scratch V((mres + 1) * nrhs * n * vsz, s);
  Scratch u(nrhs * n * (f32 ? sizeof(float2) : sizeof(double2)), s), r64(f32 ? nrhs * n * sizeof(double2) : 0, s);
  Scratch qd(b32 ? nrhs * n * sizeof(double2) : 0, s);
  Scratch A32own(f32 && A32in == nullptr ? n * n * sizeof(float2) : 0, s);
  const int np = (int)((n + 127) / 128);  // partial norm sums per vector (128-row blocks)
  const size_t hbytes = (size_t)nrhs * (mres + 1) * mres * sizeof(double2), cbytes = (size_t)nrhs * (mres + 1) * sizeof(double2);
  const int64_t ms = S > 0 ? mres / S * S : 0;  // s-step cycle length
  const size_t hsbytes = S > 0 ? (size_t)nrhs * (ms + S) * (ms + S + 1) * sizeof(double2) : 0;
  Scratch Rs(hbytes, s), Hs(std::max(hbytes, hsbytes), s), csb(nrhs * mres * sizeof(double2), s), snb(nrhs * mres * sizeof(double2), s),
      gb(cbytes, s), d1b(cbytes, s), d2b(cbytes, s), d1t(cbytes, s), d2t(cbytes, s), hcb(cbytes, s),
      abb(nrhs * sizeof(double2), s), dbl(5 * nrhs * sizeof(double), s), ints(3 * nrhs * sizeof(int32_t), s),
      part(nrhs * np * sizeof(double), s);
  // few 128-row update blocks (a single right-hand side): the basis range
  // of each is split over up to 8 blocks, so that about 256 blocks stream
  const int split = nrhs == 1 && np < 64 ? (int)std::min<int64_t>(8, (256 + np - 1) / np) : 1;
  Scratch wsb(split > 1 ? (size_t)nrhs * np * split * 256 * sizeof(double2) : 0, s);
  GmresState gs{Rs.as<double2>(),
                Hs.as<double2>(),
                csb.as<double2>(),
                snb.as<double2>(),
                gb.as<double2>(),
                d1b.as<double2>(),
                d2b.as<double2>(),
                abb.as<double2>(),
                dbl.as<double>(),
                dbl.as<double>() + nrhs,
                dbl.as<double>() + 2 * nrhs,
                dbl.as<double>() + 3 * nrhs,
                dbl.as<double>() + 4 * nrhs,
                ints.as<int32_t>(),
                ints.as<int32_t>() + nrhs,
                ints.as<int32_t>() + 2 * nrhs,
                d1t.as<double2>(),
                d2t.as<double2>(),
                hcb.as<double2>(),
                mres + 1,
                split,
                wsb.as<double2>()};
  const int64_t vstride = nrhs * n;
  const dim3 g1((unsigned)((nrhs + 63) / 64)), b1(64);
  CBFM_HIP(hipMemsetAsync(x, 0, nrhs * n * sizeof(double2), s));
  CBFM_HIP(hipMemsetAsync(gs.its, 0, nrhs * sizeof(int32_t), s));
  hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, b, n, gs.bnorm, nullptr);
  GmresResult out;
  out.its.assign(nrhs, 0);
  out.res.assign(nrhs, 1.0);
  int64_t total = 0;
  const double tol = p.tol;
  // Convergence flags go to pinned host memory every few iterations and are
  // read one check later, so the host never waits for the device inside a
  // cycle; iterations queued after the last right-hand side converged do
  // nothing (every kernel skips inactive right-hand sides).
  PinnedFlags flags(nrhs);
  auto all_done = [&](const int32_t* a) {
    return std::none_of(a, a + nrhs, [](int32_t v) { return v != 0; });
  };
  // w = A q_j for every Krylov index j, descriptors uploaded once
  const float2* A32 = A32in;
  int64_t ld32 = lda32;
  std::vector<std::vector<GemmDesc>> mv(dense && !f32 ? mres : 0);
  std::vector<std::vector<GemmDescX>> mvx(f32 ? mres : 0);
  if (f32) {
    if (A32 == nullptr) {
      hipLaunchKernelGGL(to_float_kernel, grid2(n, n), dim3(256), 0, s, A64, lda64, A32own.as<float2>(), n, n, n);
      CBFM_HIP(hipGetLastError());
      A32 = A32own.as<float2>();
      ld32 = n;
    }
    for (int64_t j = 0; j < mres; ++j) {
      GemmDescX d = gemmx(A32, 0, ld32, OP_N, V.as<float2>() + j * vstride, 0, n, OP_T, u.as<float2>(), 0, n, n, nrhs,
                          n);
      d.transC = 1;
      mvx[j].push_back(d);
    }
  } else if (dense) {
    for (int64_t j = 0; j < mres; ++j) {
      const double2* q = b32 ? qd.as<double2>() : V.as<double2>() + j * vstride;
      GemmDesc d = gemm(A64, lda64, OP_N, q, n, OP_T, u.as<double2>(), n, n, nrhs, n);
      d.transC = 1;
      mv[j].push_back(d);
    }
  } else {
    op.prepare(V.as<double2>(), vstride, u.as<double2>(), mres, nrhs, s);
  }
  const GemmPlan matvec(mv, s);
  const XGemmPlan matvec32(mvx, XG_FP32, s);
  // graph replays: one matrix-vector descriptor repointed on the device
  const bool graph = p.graph && dense && mres > 0;
  std::unique_ptr<GemmPlan> dyn;
  std::unique_ptr<XGemmPlan> dyn32;
  Scratch jdev(graph ? sizeof(int64_t) : 0, s);
  if (graph && f32) dyn32.reset(new XGemmPlan({mvx[0]}, XG_FP32, s));
  if (graph && !f32) dyn.reset(new GemmPlan({mv[0]}, s, false));
  // r = b - A x in double (A x in float for a float-only operator)
  auto residual = [&](double2* r) {
    if (A64)
      apply_op(A64, lda64, n, nrhs, x, r, s);
    else if (A32in)
      apply_op32(A32in, lda32, n, nrhs, x, r, s);
    else
      op.apply(x, r, nrhs, s);
    hipLaunchKernelGGL(sub_from_kernel, dim3((unsigned)((nrhs * n + 255) / 256)), dim3(256), 0, s, b, r, nrhs * n);
  };
  const OpMV opmv{&op};
  // s-step: a first plain cycle of S + 1 iterations gives the shifts; then
  // s-step cycles, and plain ones for good after a breakdown
  bool sstep_on = S > 0 && ms >= S, shifts_ready = false;
  std::unique_ptr<SStep> sst;
  for (;;) {
    // r = b - A x  (x = 0 on the first cycle)
    double2* r = f32 ? r64.as<double2>() : u.as<double2>();
    if (total == 0)
      CBFM_HIP(hipMemcpyAsync(r, b, nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
    else
      residual(r);
    hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, r, n, gs.nrm, nullptr);
    hipLaunchKernelGGL(cycle_init_kernel, g1, b1, 0, s, gs, mres, nrhs, tol, inner);
    if (f32 || b32)
      hipLaunchKernelGGL(scale_kernel<float2>, grid2(n, nrhs), dim3(256), 0, s, r, V.as<float2>(), n, gs.nrm,
                         qd.as<double2>());
    else
      hipLaunchKernelGGL(scale_kernel<double2>, grid2(n, nrhs), dim3(256), 0, s, r, V.as<double2>(), n, gs.nrm);
    if (all_done(flags.sync_read(gs.active, s)) || total >= p.max_iter) break;
    // an s-step cycle takes whole blocks of S iterations: fewer than S left
    // run in a plain cycle (an s-step cycle would take none and the loop
    // would make no progress)
    if (sstep_on && shifts_ready && total + S > p.max_iter) sstep_on = false;
    if (f32)
      run_cycle(matvec32, dyn32.get(), dyn32 ? dyn32->desc(0) : nullptr, jdev.as<int64_t>(), V.as<float2>(),
                u.as<float2>(), vstride, n, nrhs, mres, p.max_iter, total, gs, part.as<double>(), np, flags, x, s);
    else if (b32)
      run_cycle(matvec, dyn.get(), dyn ? dyn->desc(0) : nullptr, jdev.as<int64_t>(), V.as<float2>(), u.as<double2>(),
                vstride, n, nrhs, mres, p.max_iter, total, gs, part.as<double>(), np, flags, x, s, (const float2*)nullptr,
                qd.as<double2>());
    else if (sstep_on && !shifts_ready) {
      const int64_t m1 = std::min<int64_t>(S + 1, mres);
      GmresState g1 = gs;
      g1.ms = m1 + 1;
      CBFM_HIP(hipMemsetAsync(gs.H, 0, (size_t)nrhs * (m1 + 1) * m1 * sizeof(double2), s));
      run_cycle(matvec, (const GemmPlan*)nullptr, nullptr, jdev.as<int64_t>(), V.as<double2>(), u.as<double2>(),
                vstride, n, nrhs, m1, p.max_iter, total, g1, part.as<double>(), np, flags, x, s);
      std::vector<int32_t> its1(nrhs);
      CBFM_HIP(hipMemcpyAsync(its1.data(), gs.its, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      CBFM_HIP(hipStreamSynchronize(s));
      sst.reset(new SStep(S, n, nrhs, ms, s));
      sst->prepare_dots(V.as<double2>(), vstride, s);
      sstep_shifts(*sst, g1, m1, its1, s);
      shifts_ready = true;
    } else if (sstep_on) {
      if (run_sstep_cycle(*sst, matvec, V.as<double2>(), u.as<double2>(), vstride, p.max_iter, total, gs,
                          part.as<double>(), np, flags, x, gs.H, s))
        sstep_on = false;
    } else if (dense)
      run_cycle(matvec, dyn.get(), dyn ? dyn->desc(0) : nullptr, jdev.as<int64_t>(), V.as<double2>(),
                u.as<double2>(), vstride, n, nrhs, mres, p.max_iter, total, gs, part.as<double>(), np, flags, x, s);
    else
      run_cycle(opmv, (const OpMV*)nullptr, nullptr, jdev.as<int64_t>(), V.as<double2>(), u.as<double2>(), vstride, n,
                nrhs, mres, p.max_iter, total, gs, part.as<double>(), np, flags, x, s, op.xbasis());
    if (total >= p.max_iter) break;
  }
  CBFM_HIP(hipMemcpyAsync(out.its.data(), gs.its, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  // true relative residual
  {
    double2* r = f32 ? r64.as<double2>() : u.as<double2>();
    residual(r);
    hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, r, n, gs.nrm, nullptr);
    std::vector<double> rn(nrhs), bn(nrhs);
    CBFM_HIP(hipMemcpyAsync(rn.data(), gs.nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    CBFM_HIP(hipMemcpyAsync(bn.data(), gs.bnorm, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    CBFM_HIP(hipStreamSynchronize(s));
    for (int64_t q = 0; q < nrhs; ++q) {
      out.res[q] = bn[q] > 0 ? rn[q] / bn[q] : 0.0;
      if (out.res[q] > tol) out.noconv = true;
    }
  }
  return out;
}

void permute_halves(const double2* in, double2* out, const int32_t* perm, int64_t ne, int64_t nv, int forward,
                    hipStream_t s) {
  hipLaunchKernelGGL(permute_kernel, grid2(ne, nv), dim3(256), 0, s, in, out, perm, ne, nv, forward);
  CBFM_HIP(hipGetLastError());
}

void rcs_compute(const cbfm_mesh_s* m, const cbfm_medium* med, const double2* jfinal, const double* inc, int64_t nrhs,
                 const double* dirs, int64_t ndir, double* rcs, hipStream_t s) {
  const MeshHost& h = m->h;
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
  fa.ne = h.ne;
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
  CBFM_HIP(hipStreamSynchronize(s));
}

// v_r = (C^JM)^H v for nrhs tested incident fields v (internal order, nrhs x 2ne)
void project_rhs(const cbfm_mesh_s* m, cbfm_cbf_s* c, const double2* vint, int64_t nrhs, double2* b, hipStream_t s) {
  const MeshHost& h = m->h;
  const int64_t ne = h.ne, NL = c->NL, n = 2 * NL;
  std::vector<GemmDesc> ds;
  for (int a = 0; a < h.nblocks; ++a) {
    const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], r0 = h.cell_off[a];
    // [v_r]_J-part = (C^J_a)^H v^E_a,  [v_r]_M-part = (C^M_a)^H v^H_a  (per vector: v . conj(C))
    ds.push_back(gemm(vint + r0, 2 * ne, OP_N, c->CJ.as<double2>() + c->coff[a], c->L[a], OP_R, b + c->off[a], n, nrhs,
                      c->L[a], Na));
    ds.push_back(gemm(vint + ne + r0, 2 * ne, OP_N, c->CM.as<double2>() + c->coff[a], c->L[a], OP_R,
                      b + NL + c->off[a], n, nrhs, c->L[a], Na));
  }
  zgemm_batched(ds, s);
}

// j = C^MJ j_CBF (internal order, nrhs x 2ne)
void expand_cbf(const cbfm_mesh_s* m, cbfm_cbf_s* c, const double2* jc, int64_t nrhs, double2* jint, hipStream_t s) {
  const MeshHost& h = m->h;
  const int64_t ne = h.ne, NL = c->NL, n = 2 * NL;
  std::vector<GemmDesc> ds;
  for (int a = 0; a < h.nblocks; ++a) {
    const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], r0 = h.cell_off[a];
    // alpha^M_a = C^M_a beta^M_a, alpha^J_a = C^J_a beta^J_a  (per vector: beta . C^T)
    ds.push_back(gemm(jc + c->off[a], n, OP_N, c->CM.as<double2>() + c->coff[a], c->L[a], OP_T, jint + r0, 2 * ne, nrhs,
                      Na, c->L[a]));
    ds.push_back(gemm(jc + NL + c->off[a], n, OP_N, c->CJ.as<double2>() + c->coff[a], c->L[a], OP_T, jint + ne + r0,
                      2 * ne, nrhs, Na, c->L[a]));
  }
  zgemm_batched(ds, s);
}

// Flexible GMRES with the paper's inexact CMP: each Krylov vector q_j is
// preconditioned by an inner GMRES solve z_j ~ (G^CBF)^{-1} q_j (diagonal
// preconditioner D^CBF, relative residual inner_tol), the product is
// w = Z_r z_j, and the iterate is x = sum z_j y_j: j_CBF itself.
class FlexCmpOp : public KrylovOp {
 public:
  FlexCmpOp(const double2* Zr, int64_t ldz, cbfm_cbf_s* c, double inner_tol, int64_t n)
      : Zr_(Zr), ldz_(ldz), c_(c), tol_(inner_tol), n_(n) {}
  void prepare(const double2* V, int64_t vstride, double2* w, int64_t mres, int64_t nrhs, hipStream_t s) override {
    V_ = V;
    vstride_ = vstride;
    nrhs_ = nrhs;
    Zb_.reset(new Scratch((size_t)mres * vstride * sizeof(double2), s));
    std::vector<std::vector<GemmDesc>> g(mres);
    for (int64_t j = 0; j < mres; ++j) {
      GemmDesc d = gemm(Zr_, ldz_, OP_N, Zb_->as<double2>() + j * vstride, n_, OP_T, w, n_, n_, nrhs, n_);
      d.transC = 1;
      g[j].push_back(d);
    }
    plan_.reset(new GemmPlan(g, s, false));
  }
  void launch(int64_t j, hipStream_t q) const override {
    cmp_inner_apply(c_, nrhs_, V_ + j * vstride_, Zb_->as<double2>() + j * vstride_, tol_, q);
    plan_->launch((size_t)j, q);
  }
  void apply(const double2* x, double2* r, int64_t nrhs, hipStream_t s) const override {
    apply_op(Zr_, ldz_, n_, nrhs, x, r, s);
  }
  const double2* xbasis() const override { return Zb_ ? Zb_->as<double2>() : nullptr; }

 private:
  const double2* Zr_;
  int64_t ldz_;
  cbfm_cbf_s* c_;
  double tol_;
  int64_t n_, nrhs_ = 0, vstride_ = 0;
  const double2* V_ = nullptr;
  std::unique_ptr<Scratch> Zb_;
  std::unique_ptr<GemmPlan> plan_;
};

// out[c][i] = in[c][(i + NL) mod 2NL]: the two halves of each vector swapped
__global__ void swap_halves_kernel(const double2* __restrict__ in, double2* __restrict__ out, int64_t NL, int64_t nv,
                                   int64_t ldi, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (i >= 2 * NL || c >= nv) return;
  out[c * ldo + i] = in[c * ldi + (i < NL ? i + NL : i - NL)];
}

}  // namespace cbfm

using namespace cbfm;

extern "C" cbfm_status cbfm_solve(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, const void* Zr_v, int64_t ldz,
                                  const double* inc, int64_t nrhs, const cbfm_solver_params* prm, void* j_dev,
                                  int32_t* iters, double* relres, const double* dirs, int64_t ndir, double* rcs,
                                  void* stream) {
  bool noconv = false;
  cbfm_status st = guarded([&] {
    CBFM_REQUIRE(m && c && Zr_v && inc && prm, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(c->mesh == m, CBFM_E_STATE, "CBF set belongs to another mesh");
    CBFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, CBFM_E_ARG, "nrhs out of range");
    CBFM_REQUIRE(ldz >= 2 * c->NL, CBFM_E_ARG, "ldz < N_CBF");
    CBFM_REQUIRE(prm->tol > 0 && prm->max_iter >= 1 && prm->restart >= 1, CBFM_E_ARG, "bad solver parameters");
    CBFM_REQUIRE(prm->use_cmp >= 0 && prm->use_cmp <= 2, CBFM_E_ARG, "use_cmp must be 0, 1 or 2");
    CBFM_REQUIRE(prm->cmp_mode == CBFM_CMP_EXACT || prm->cmp_mode == CBFM_CMP_INNER_GMRES, CBFM_E_ARG,
                 "unknown CMP mode");
    const bool flexible = prm->use_cmp == 1 && prm->cmp_mode == CBFM_CMP_INNER_GMRES;
    CBFM_REQUIRE(!flexible || (prm->inner_fp32 == 0 && prm->use_graph == 0 && prm->basis_fp32 == 0), CBFM_E_ARG,
                 "the inexact CMP runs double Krylov cycles with a double basis and without graphs");
    CBFM_REQUIRE(prm->inner_fp32 == 0 || prm->basis_fp32 == 0, CBFM_E_ARG,
                 "inner_fp32 and basis_fp32 are two different forms");
    CBFM_REQUIRE(prm->sstep == 0 || ((prm->sstep == 4 || prm->sstep == 8) && !flexible && prm->inner_fp32 == 0 &&
                                     prm->basis_fp32 == 0 && prm->use_graph == 0),
                 CBFM_E_ARG, "sstep is 0, 4 or 8, with double cycles, the exact CMP and no graphs");
    CBFM_REQUIRE(prm->block == 0 || (prm->block >= 1 && prm->block <= 32 && !flexible && prm->inner_fp32 == 0 && prm->basis_fp32 == 0 &&
                                     prm->use_graph == 0 && prm->sstep == 0),
                 CBFM_E_ARG, "block is 0 to 32, with double cycles, the exact CMP, no graphs and no s-step cycles");
    CBFM_REQUIRE(prm->inner_tol >= 0 && prm->inner_tol < 1, CBFM_E_ARG, "inner_tol outside [0, 1)");
    CBFM_REQUIRE(!flexible || (prm->cmp_inner_tol >= 0 && prm->cmp_inner_tol < 1), CBFM_E_ARG,
                 "cmp_inner_tol outside [0, 1)");
    CBFM_REQUIRE(dirs == nullptr || ndir >= 1, CBFM_E_ARG, "ndir must be >= 1 with dirs");
    const Media md = make_media(med);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MeshHost& h = m->h;
    const int64_t ne = h.ne, NL = c->NL, n = 2 * NL;
    const double2* Zr = static_cast<const double2*>(Zr_v);
    // ---- right-hand sides and their projection
    Scratch dinc(nrhs * 6 * sizeof(double), s);
    CBFM_HIP(hipMemcpyAsync(dinc.p, inc, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, s));
    Scratch v(nrhs * 2 * ne * sizeof(double2), s), vint(nrhs * 2 * ne * sizeof(double2), s);
    rhs_launch(m, md, med->eta0, dinc.as<double>(), nrhs, v.p, s);
    permute_halves(v.as<double2>(), vint.as<double2>(), m->perm.as<int32_t>(), ne, nrhs, 1, s);
    Scratch b(nrhs * n * sizeof(double2), s);
    project_rhs(m, c, vint.as<double2>(), nrhs, b.as<double2>(), s);
    // ---- operator.  use_cmp 1: right-preconditioned A = Z_r (G^CBF)^{-1},
    // formed once, with (G^CBF)^{-1} = blkdiag(-(B^{-1})^H, B^{-1}).
    // use_cmp 2 (T-diagonal CBFM, Sec. IV-A): (C^JM)^H Z_t C^JM = Z_r with
    // its two column halves swapped, solved without preconditioner.
    const double2* Aop = Zr;
    int64_t lda = ldz;
    Scratch Ap(prm->use_cmp && !flexible ? n * n * sizeof(double2) : 0, s);
    if (flexible) {
      // (no operator formed: flexible GMRES applies Z_r after each inner solve)
    } else if (prm->use_cmp == 1) {
      const double2* Bi = cmp_inverse(c, s);
      std::vector<GemmDesc> ds;
      if (c->blockdiag) {  // B^{-1} block-diagonal: each cell's columns take its own block
        for (int a = 0; a < h.nblocks; ++a) {
          const int64_t o = c->off[a], La = c->L[a];
          const double2* Ba = Bi + o * NL + o;
          ds.push_back(gemm(Zr + o, ldz, OP_N, Ba, NL, OP_C, Ap.as<double2>() + o, n, n, La, La, -1.0));
          ds.push_back(gemm(Zr + NL + o, ldz, OP_N, Ba, NL, OP_N, Ap.as<double2>() + NL + o, n, n, La, La));
        }
      } else {
        ds.push_back(gemm(Zr, ldz, OP_N, Bi, NL, OP_C, Ap.as<double2>(), n, n, NL, NL, -1.0));
        ds.push_back(gemm(Zr + NL, ldz, OP_N, Bi, NL, OP_N, Ap.as<double2>() + NL, n, n, NL, NL));
      }
      zgemm_batched(ds, s);
      Aop = Ap.as<double2>();
      lda = n;
    } else if (prm->use_cmp == 2) {
      // row r of Z_r Pi: row r of Z_r with its halves swapped
      hipLaunchKernelGGL(swap_halves_kernel, grid2(n, n), dim3(256), 0, s, Zr, Ap.as<double2>(), NL, n, ldz, n);
      CBFM_HIP(hipGetLastError());
      Aop = Ap.as<double2>();
      lda = n;
    }
    GmresSpec sp;
    sp.tol = prm->tol;
    sp.max_iter = prm->max_iter;
    sp.restart = prm->restart;
    sp.f32 = prm->inner_fp32 != 0;
    sp.inner_tol = prm->inner_tol;
    sp.graph = prm->use_graph != 0;
    sp.basis32 = prm->basis_fp32 != 0;
    sp.sstep = prm->sstep;
    sp.block = prm->block;
    Scratch x(nrhs * n * sizeof(double2), s);
    DenseOp dop(Aop, lda, nullptr, 0);
    FlexCmpOp fop(Zr, ldz, c, prm->cmp_inner_tol > 0 ? prm->cmp_inner_tol : 1e-5, n);
    const GmresResult res =
        gmres_run(flexible ? (KrylovOp&)fop : (KrylovOp&)dop, n, nrhs, b.as<double2>(), x.as<double2>(), sp, s);
    noconv = res.noconv;
    // j_CBF = G^{-1} x (CMP), x itself (flexible: the iterate is j_CBF), or
    // Pi x (T-diagonal: [J CBFs; M CBFs] -> [M; J]); j = C^MJ j_CBF
    double2* jc = x.as<double2>();
    Scratch jsw(prm->use_cmp == 2 ? nrhs * n * sizeof(double2) : 0, s);
    if (prm->use_cmp == 1 && !flexible) cmp_apply_dev(c, nrhs, jc, s);
    if (prm->use_cmp == 2) {
      hipLaunchKernelGGL(swap_halves_kernel, grid2(n, nrhs), dim3(256), 0, s, jc, jsw.as<double2>(), NL, nrhs, n, n);
      CBFM_HIP(hipGetLastError());
      jc = jsw.as<double2>();
    }
    Scratch jint(nrhs * 2 * ne * sizeof(double2), s), jout(nrhs * 2 * ne * sizeof(double2), s);
    expand_cbf(m, c, jc, nrhs, jint.as<double2>(), s);
    double2* jfinal = j_dev ? static_cast<double2*>(j_dev) : jout.as<double2>();
    permute_halves(jint.as<double2>(), jfinal, m->perm.as<int32_t>(), ne, nrhs, 0, s);
    if (rcs) rcs_compute(m, med, jfinal, inc, nrhs, dirs, ndir, rcs, s);
    CBFM_HIP(hipStreamSynchronize(s));
    if (iters) std::memcpy(iters, res.its.data(), nrhs * sizeof(int32_t));
    if (relres) std::memcpy(relres, res.res.data(), nrhs * sizeof(double));
    if (noconv) set_error("GMRES did not reach the tolerance for every right-hand side");
  });
  return st != CBFM_OK ? st : (noconv ? CBFM_E_NOCONV : CBFM_OK);
}
