// PMCHWT Galerkin fill on gfx950 (paper Sec. II-B, entries [K_i]_mn and
// [T_i]_mn and the block matrix Z).
//
// Regular pairs: one lane per (test triangle P, source triangle Q) pair,
// 7 x 7 point pairs, both media.  Per pair the kernel accumulates, with
// coordinates taken relative to each triangle's own centroid (r~ = r - c_P,
// r~' = r' - c_Q, d = c_P - c_Q, so r - r' = r~ + d - r~'):
//   T part (per medium): I0 = S G, Ir = S G r~, Irq = S G r~', Irr = S G r~.r~'
//   K part (media summed, g = g1 + g2): S0 = S g r~.(X x r~'),
//     SA = S g X x r~', SB = S g r~ x X, SC = S g X        (X = r - r')
// with S the weighted double sum, and forms the 3 x 3 local blocks
//   T_i[a,b] = c_a c_b ( (j k_i / 4) (Irr - q~_b.Ir - p~_a.Irq + p~_a.q~_b I0)
//                        - (j / k_i) I0 )
//   K[a,b]   = -(c_a c_b / 4) ( S0 - p~_a.SA - q~_b.SB + p~_a.(SC x q~_b) )
// (c_a = s_a l_a, p_a / q_b the free vertices).  Every term is of the size
// of the result, so no cancellation grows with the distance of the pair.
//
// Near pairs: FP64, 7-point outer rule (one thread per pair and outer point
// for the inner integrals, one thread per pair for the contraction); on the source
// triangle the 1/R - k^2 R/2 part of 4 pi G and the 1/R^3 + k^2/(2R) part
// of -4 pi g are integrated in closed form (potentials of a flat triangle),
// the bounded remainders by the 7-point rule.  K of a coplanar pair is 0.
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace cbfm {

struct FillConsts {
  double w[7];
  double wq[7][7];            // w_k w_l / (4 pi): point-pair weights of the regular rule
  float wqf[7][7];
  double bary[7][3];
  double k1, k2r, k2i;
  double rev1, rev2;          // k / (2 pi): phase in revolutions (FP32 path)
  // output op o in {1, 2}: op_o = c_a c_b sum_i (A[o][i] X_i + B[o][i] I0_i)
  double A[2][2][2], B[2][2][2];  // [op][medium][re/im]
  // near kernel: per-medium j k_i and 1/k_i^2 and the output weights e[o][i]
  double jk[2][2], ik2[2][2], e[2][2][2];
  double ksq_re, ksq_im;      // k1^2 + k2^2
};

template <typename R>
struct cx {
  R re, im;
};

Media make_media(const cbfm_medium* med) {
  CBFM_REQUIRE(med != nullptr, CBFM_E_ARG, "medium is NULL");
  CBFM_REQUIRE(med->k0 > 0 && std::isfinite(med->k0) && med->eta0 > 0, CBFM_E_ARG,
               "need k0 > 0 and eta0 > 0");
  const std::complex<double> eps(med->eps_re, med->eps_im), mu(med->mu_re, med->mu_im);
  CBFM_REQUIRE(std::abs(eps) > 0 && std::abs(mu) > 0, CBFM_E_ARG, "eps_r and mu_r must be nonzero");
  Media m;
  m.k1 = med->k0;
  const std::complex<double> k2 = med->k0 * std::sqrt(eps * mu);
  m.k2r = k2.real();
  m.k2i = k2.imag();
  CBFM_REQUIRE(m.k2i <= 0 && m.k2r > 0, CBFM_E_ARG, "interior wavenumber must have Re k > 0, Im k <= 0");
  m.eta1 = med->eta0;
  m.eta2 = med->eta0 * std::sqrt(mu / eps);
  return m;
}

static FillConsts make_consts(const Media& md, int layout) {
  FillConsts fc{};
  const double s15 = std::sqrt(15.0);
  const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
  const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
  const double W[7] = {9.0 / 40.0, wa, wa, wa, wb, wb, wb};
  const double B[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {1 - 2 * a, a, a}, {a, 1 - 2 * a, a},
                          {a, a, 1 - 2 * a},           {1 - 2 * b, b, b}, {b, 1 - 2 * b, b},
                          {b, b, 1 - 2 * b}};
  for (int k = 0; k < 7; ++k) {
    fc.w[k] = W[k];
    for (int i = 0; i < 3; ++i) fc.bary[k][i] = B[k][i];
    for (int l = 0; l < 7; ++l) {
      fc.wq[k][l] = W[k] * W[l] * (0.25 / M_PI);
      fc.wqf[k][l] = (float)fc.wq[k][l];
    }
  }
  fc.k1 = md.k1;
  fc.k2r = md.k2r;
  fc.k2i = md.k2i;
  fc.rev1 = md.k1 / (2 * M_PI);
  fc.rev2 = md.k2r / (2 * M_PI);
  using C = std::complex<double>;
  const C j(0, 1);
  const C k[2] = {C(md.k1, 0), C(md.k2r, md.k2i)};
  C e[2][2];  // [op][medium]
  if (layout == CBFM_LAYOUT_OPS3) {
    e[0][0] = md.eta1;
    e[0][1] = md.eta2;
    e[1][0] = 1.0 / md.eta1;
    e[1][1] = 1.0 / md.eta2;
  } else {
    e[0][0] = 1;
    e[0][1] = 0;
    e[1][0] = 0;
    e[1][1] = 1;
  }
  for (int o = 0; o < 2; ++o)
    for (int i = 0; i < 2; ++i) {
      const C alpha = j * k[i] / 4.0, beta = -j / k[i];
      const C A = e[o][i] * alpha, Bc = e[o][i] * beta;
      fc.A[o][i][0] = A.real();
      fc.A[o][i][1] = A.imag();
      fc.B[o][i][0] = Bc.real();
      fc.B[o][i][1] = Bc.imag();
      fc.e[o][i][0] = e[o][i].real();
      fc.e[o][i][1] = e[o][i].imag();
    }
  for (int i = 0; i < 2; ++i) {
    const C jk = j * k[i], ik2 = 1.0 / (k[i] * k[i]);
    fc.jk[i][0] = jk.real();
    fc.jk[i][1] = jk.imag();
    fc.ik2[i][0] = ik2.real();
    fc.ik2[i][1] = ik2.imag();
  }
  const C ksq = k[0] * k[0] + k[1] * k[1];
  fc.ksq_re = ksq.real();
  fc.ksq_im = ksq.imag();
  return fc;
}

// ------------------------------------------------------------- phase helpers
// sin and cos of 2 pi x, x in revolutions: x = n / 2 + f with n = rint(2 x),
// |f| <= 1/4 (the subtraction is exact), then with u = f^2
//   sin(2 pi f) = f S(u),  cos(2 pi f) = C(u),
// S and C polynomials of degree 8 in u on [0, 1/16]: near-minimax fits
// (Chebyshev interpolation of sin(2 pi sqrt u) / sqrt u and
// cos(2 pi sqrt u) at 9 nodes, computed in 50-digit arithmetic; fit error
// 1.3e-18 and 3.9e-18, under a quarter ulp of the results, so that the
// Horner evaluation in FP64 stays within an ulp).  A half turn only flips
// both signs, applied to the sign bits.  The phases here are small
// multiples of 2 pi (k R over a scatterer), where this reduction is exact
// enough.  17 FMAs, 3 products and a rint for the pair of values.
__device__ __forceinline__ void sincos_rev(double x, double& s, double& c) {
  const double q = rint(2.0 * x);
  const double f = fma(-0.5, q, x);
  const int flip = ((int)q & 1) << 31;
  const double u = f * f;
  double ps = 0.10089695501646812;
  ps = fma(ps, u, -0.71773379214134536);
  ps = fma(ps, u, 3.8199280942271643);
  ps = fma(ps, u, -15.094641676117901);
  ps = fma(ps, u, 42.058693925428685);
  ps = fma(ps, u, -76.705859752824921);
  ps = fma(ps, u, 81.605249276073621);
  ps = fma(ps, u, -41.341702240399755);
  ps = fma(ps, u, 6.2831853071795862);
  const double sn = f * ps;
  double pc = 0.2719458494999813;
  pc = fma(pc, u, -1.7132184107005932);
  pc = fma(pc, u, 7.9034624920850973);
  pc = fma(pc, u, -26.426254066690255);
  pc = fma(pc, u, 60.244641313160407);
  pc = fma(pc, u, -85.456817205980613);
  pc = fma(pc, u, 64.939394022663947);
  pc = fma(pc, u, -19.739208802178705);
  const double cs = fma(pc, u, 1.0);
  s = __hiloint2double(__double2hiint(sn) ^ flip, __double2loint(sn));
  c = __hiloint2double(__double2hiint(cs) ^ flip, __double2loint(cs));
}
__device__ __forceinline__ void phase(double /*x_rad*/, double x_rev, double& s, double& c) { sincos_rev(x_rev, s, c); }
__device__ __forceinline__ void phase(float /*x_rad*/, float x_rev, float& s, float& c) {
  // hardware sine/cosine take the angle in revolutions
  const float f = __builtin_amdgcn_fractf(x_rev);
  s = __builtin_amdgcn_sinf(f);
  c = __builtin_amdgcn_cosf(f);
}
// 1 / sqrt(x): the hardware estimate (relative error about 5e-8 on gfx950)
// refined by one Newton step y <- y + y (1 - x y^2) / 2, which squares the
// error (a few 1e-15; the residual is formed with an FMA).
__device__ __forceinline__ double rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double r = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, r, y);
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double expo(double x) { return exp(x); }
__device__ __forceinline__ float expo(float x) { return __expf(x); }

// ------------------------------------------------------------- regular kernel
__device__ __forceinline__ double pair_weight(const FillConsts& fc, int k, int l, double) { return fc.wq[k][l]; }
__device__ __forceinline__ float pair_weight(const FillConsts& fc, int k, int l, float) { return fc.wqf[k][l]; }

// The 3 x 3 local blocks of the three output operators for test triangle P
// and source triangle Q, written at o0 (row stride ldl, operator stride
// op_stride).  P is the same on every lane of the wavefront (one row
// triangle per block): its quadrature points are read into scalar
// registers, and the loop over them is the inner one.  The outer loop runs
// over the lane's own source points r~'_l, so that only one of them (and
// e_l = d - r~'_l, with X = r~_k + e_l) is held per lane.  Per source point
// the inner sums over the test points are
//   A0 = S_k G,  B0 = S_k g,  B1 = S_k g r~_k,
// and the moments follow from them and the lane's vectors:
//   S_k g X = B1 + e_l B0,   S_k g X x r~' = (S_k g X) x r~',
//   S_k g r~ x X = B1 x e_l, S_k g r~.(X x r~') = B1.(e_l x r~')
// (r~ x r~ = 0 and r~.(r~ x r~') = 0 drop out exactly); Ir and Irr take
// the test point itself and are summed in the inner loop.
template <typename R, bool LOSSY>
__device__ __forceinline__ void regular_pair(const TriTab<R>& tab, int32_t P, int32_t Q, const FillConsts& fc,
                                             cx<R>* __restrict__ o0, int64_t op_stride, int64_t ldl) {
  const int64_t nt = tab.nt;
  P = __builtin_amdgcn_readfirstlane(P);

  const R d[3] = {(R)(tab.cen[0][P] - tab.cen[0][Q]), (R)(tab.cen[1][P] - tab.cen[1][Q]),
                  (R)(tab.cen[2][P] - tab.cen[2][Q])};
  const R k1 = (R)fc.k1, k2r = (R)fc.k2r, k2i = (R)fc.k2i;
  const R rev1 = (R)fc.rev1, rev2 = (R)fc.rev2;

  cx<R> I0[2] = {}, Ir[2][3] = {}, Irq[2][3] = {}, Irr[2] = {};
  cx<R> S0 = {}, SA[3] = {}, SB[3] = {}, SC[3] = {};

#pragma unroll 1
  for (int l = 0; l < 7; ++l) {
    const R rq[3] = {tab.q[0][l * nt + Q], tab.q[1][l * nt + Q], tab.q[2][l * nt + Q]};
    const R e[3] = {d[0] - rq[0], d[1] - rq[1], d[2] - rq[2]};
    cx<R> A0[2] = {}, B0 = {}, B1[3] = {};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const R rk[3] = {tab.q[0][k * nt + P], tab.q[1][k * nt + P], tab.q[2][k * nt + P]};
      const R x0 = rk[0] + e[0], x1 = rk[1] + e[1], x2 = rk[2] + e[2];
      const R R2 = x0 * x0 + x1 * x1 + x2 * x2;
      const R iR = rsq(R2);
      const R Rl = R2 * iR;
      const R f = pair_weight(fc, k, l, R(0)) * iR;  // w_k w_l / (4 pi R)
      const R t = iR * iR;
      // exterior medium
      const R ph1 = k1 * Rl;
      R s1, c1;
      phase(ph1, rev1 * Rl, s1, c1);
      const cx<R> G1 = {c1 * f, -s1 * f};
      // interior medium
      const R ph2 = k2r * Rl;
      R s2, c2;
      phase(ph2, rev2 * Rl, s2, c2);
      R f2 = f;
      R u = (R)1;
      if (LOSSY) {
        f2 = f * expo(k2i * Rl);
        u = (R)1 - k2i * Rl;
      }
      const cx<R> G2 = {c2 * f2, -s2 * f2};
      // g = -G (1 + j k R) / R^2, summed over media (weights included)
      const cx<R> g = {-((G1.re - ph1 * G1.im) + (u * G2.re - ph2 * G2.im)) * t,
                       -((G1.im + ph1 * G1.re) + (u * G2.im + ph2 * G2.re)) * t};
      A0[0].re += G1.re;
      A0[0].im += G1.im;
      A0[1].re += G2.re;
      A0[1].im += G2.im;
      B0.re += g.re;
      B0.im += g.im;
      const R rr = rk[0] * rq[0] + rk[1] * rq[1] + rk[2] * rq[2];
      Irr[0].re += G1.re * rr;
      Irr[0].im += G1.im * rr;
      Irr[1].re += G2.re * rr;
      Irr[1].im += G2.im * rr;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R q = rk[c];
        Ir[0][c].re += G1.re * q;
        Ir[0][c].im += G1.im * q;
        Ir[1][c].re += G2.re * q;
        Ir[1][c].im += G2.im * q;
        B1[c].re += g.re * q;
        B1[c].im += g.im * q;
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      I0[m].re += A0[m].re;
      I0[m].im += A0[m].im;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Irq[m][c].re += A0[m].re * rq[c];
        Irq[m][c].im += A0[m].im * rq[c];
      }
    }
    // K moments of this source point
    cx<R> X[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      X[c].re = B1[c].re + e[c] * B0.re;  // S_k g X
      X[c].im = B1[c].im + e[c] * B0.im;
    }
    R ex[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      ex[c] = e[c1] * rq[c2] - e[c2] * rq[c1];                  // e_l x r~'
      SC[c].re += X[c].re;
      SC[c].im += X[c].im;
      SA[c].re += X[c1].re * rq[c2] - X[c2].re * rq[c1];         // (S_k g X) x r~'
      SA[c].im += X[c1].im * rq[c2] - X[c2].im * rq[c1];
      SB[c].re += B1[c1].re * e[c2] - B1[c2].re * e[c1];         // B1 x e_l
      SB[c].im += B1[c1].im * e[c2] - B1[c2].im * e[c1];
    }
    S0.re += B1[0].re * ex[0] + B1[1].re * ex[1] + B1[2].re * ex[2];
    S0.im += B1[0].im * ex[0] + B1[1].im * ex[1] + B1[2].im * ex[2];
  }

  // epilogue: 3 x 3 local blocks of K, op1, op2
  R pv[3][3], qv[3][3], ca[3], cb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ca[a] = tab.c[a * nt + P];
    cb[a] = tab.c[a * nt + Q];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv[a][c] = tab.v[c][a * nt + P];
      qv[a][c] = tab.v[c][a * nt + Q];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R* p = pv[a];
    const cx<R> pSA = {p[0] * SA[0].re + p[1] * SA[1].re + p[2] * SA[2].re,
                       p[0] * SA[0].im + p[1] * SA[1].im + p[2] * SA[2].im};
    cx<R> pIrq[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      pIrq[m].re = p[0] * Irq[m][0].re + p[1] * Irq[m][1].re + p[2] * Irq[m][2].re;
      pIrq[m].im = p[0] * Irq[m][0].im + p[1] * Irq[m][1].im + p[2] * Irq[m][2].im;
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const R* q = qv[b];
      const R cab = ca[a] * cb[b];
      // K
      cx<R> SCxq[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        SCxq[c].re = SC[c1].re * q[c2] - SC[c2].re * q[c1];
        SCxq[c].im = SC[c1].im * q[c2] - SC[c2].im * q[c1];
      }
      const R kre = S0.re - pSA.re - (q[0] * SB[0].re + q[1] * SB[1].re + q[2] * SB[2].re) +
                    (p[0] * SCxq[0].re + p[1] * SCxq[1].re + p[2] * SCxq[2].re);
      const R kim = S0.im - pSA.im - (q[0] * SB[0].im + q[1] * SB[1].im + q[2] * SB[2].im) +
                    (p[0] * SCxq[0].im + p[1] * SCxq[1].im + p[2] * SCxq[2].im);
      const R kf = (R)(-0.25) * cab;
      o0[a * ldl + b] = cx<R>{kf * kre, kf * kim};
      // T per medium: X_m = Irr - q.Ir - p.Irq + (p.q) I0
      const R pq = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
      cx<R> X[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        X[m].re = Irr[m].re - (q[0] * Ir[m][0].re + q[1] * Ir[m][1].re + q[2] * Ir[m][2].re) -
                  pIrq[m].re + pq * I0[m].re;
        X[m].im = Irr[m].im - (q[0] * Ir[m][0].im + q[1] * Ir[m][1].im + q[2] * Ir[m][2].im) -
                  pIrq[m].im + pq * I0[m].im;
      }
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        R re = 0, im = 0;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const R Ar = (R)fc.A[o][m][0], Ai = (R)fc.A[o][m][1];
          const R Br = (R)fc.B[o][m][0], Bi = (R)fc.B[o][m][1];
          re += Ar * X[m].re - Ai * X[m].im + Br * I0[m].re - Bi * I0[m].im;
          im += Ar * X[m].im + Ai * X[m].re + Br * I0[m].im + Bi * I0[m].re;
        }
        o0[(o + 1) * op_stride + a * ldl + b] = cx<R>{cab * re, cab * im};
      }
    }
  }
}

template <typename R, bool LOSSY>
__global__ void __launch_bounds__(256, 2) fill_regular_kernel(
    TriTab<R> tab, const int32_t* __restrict__ rowTris, const int32_t* __restrict__ colTris,
    int64_t nct, FillConsts fc, cx<R>* __restrict__ out, int64_t op_stride, int64_t ldl) {
  const int64_t i = blockIdx.y;
  const int64_t jq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jq >= nct) return;
  regular_pair<R, LOSSY>(tab, rowTris[i], colTris[jq], fc, out + (3 * i) * ldl + 3 * jq, op_stride, ldl);
}

// Many fills (scatterers of any size, each with its own medium) in one
// persistent launch: a work item is one row triangle of one job against 256
// of its columns; blocks stride over the items of all jobs.
template <typename R>
struct FillJob {
  TriTab<R> tab;
  FillConsts fc;
  const int32_t* rowTris;
  const int32_t* colTris;
  int64_t nct, op_stride, ldl;
  cx<R>* out;
  int32_t lossy;
  int64_t item0;  // first work item of the job
};

template <typename R>
__global__ void __launch_bounds__(256, 2) fill_regular_batch_kernel(const FillJob<R>* __restrict__ jobs, int njobs,
                                                                     int64_t total) {
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].item0 <= it)
        lo = mid;
      else
        hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const FillJob<R>& J = jobs[lo];
    const int64_t local = it - J.item0, chunks = (J.nct + 255) / 256;
    const int64_t i = local / chunks, jq = (local % chunks) * 256 + threadIdx.x;
    if (jq >= J.nct) continue;
    cx<R>* o0 = J.out + (3 * i) * J.ldl + 3 * jq;
    if (J.lossy)
      regular_pair<R, true>(J.tab, J.rowTris[i], J.colTris[jq], J.fc, o0, J.op_stride, J.ldl);
    else
      regular_pair<R, false>(J.tab, J.rowTris[i], J.colTris[jq], J.fc, o0, J.op_stride, J.ldl);
  }
}

// ------------------------------------------------------------- near kernel
struct cd {
  double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }

// e^{-j k R} for k = kr + j ki
__device__ __forceinline__ cd cexpm(double kr, double ki, double R) {
  double s, c;
  sincos(kr * R, &s, &c);
  const double a = exp(ki * R);
  return {a * c, -a * s};
}

// 4 pi G - (1/R - k^2 R / 2), divided by 4 pi; limit -jk / (4 pi) at R = 0
__device__ cd Gr_rem(double kr, double ki, double R) {
  const double i4p = 0.25 / M_PI;
  if (R == 0.0) return {ki * i4p, -kr * i4p};  // -j k
  const cd e = cexpm(kr, ki, R);
  const cd k2 = {kr * kr - ki * ki, 2 * kr * ki};
  cd v = cscale({e.re - 1.0, e.im}, 1.0 / R);
  v = cadd(v, cscale(k2, 0.5 * R));
  return cscale(v, i4p);
}

// g + (1/R^3 + k^2/(2R)) / (4 pi); limit j k^3/(12 pi) at R = 0
__device__ cd gr_rem(double kr, double ki, double R) {
  const double i4p = 0.25 / M_PI;
  const cd k = {kr, ki};
  const cd k2 = cmul(k, k);
  if (R == 0.0) {
    const cd k3 = cmul(k2, k);
    return cscale({-k3.im, k3.re}, i4p / 3.0);  // j k^3 / 3
  }
  const cd e = cexpm(kr, ki, R);
  const cd one_jkR = {1.0 - ki * R, kr * R};  // 1 + j k R
  cd v = cmul(one_jkR, e);
  v = {-v.re + 1.0 + 0.5 * k2.re * R * R, -v.im + 0.5 * k2.im * R * R};
  return cscale(v, i4p / (R * R * R));
}

struct Pot {
  double Im1, I1, Vm1[3], V1[3], Gm3[3];
};

// Closed-form integrals over the triangle (a0, a1, a2) for the point r.
__device__ void tri_potentials(const double r[3], const double v[3][3], Pot& o) {
  double e1[3], e2[3], n[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = v[1][c] - v[0][c];
    e2[c] = v[2][c] - v[0][c];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int c = 0; c < 3; ++c) n[c] /= nn;
  const double d = (r[0] - v[0][0]) * n[0] + (r[1] - v[0][1]) * n[1] + (r[2] - v[0][2]) * n[2];
  const double rho[3] = {r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2]};
  const double ad = fabs(d);
  double sum_t0f = 0, sum_beta = 0, sum_t0F1 = 0, pm1[3] = {0, 0, 0}, p1[3] = {0, 0, 0},
         uf[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const double* a = v[i];
    const double* b = v[(i + 1) % 3];
    double t[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double L = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int c = 0; c < 3; ++c) t[c] /= L;
    const double u[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
    const double am[3] = {a[0] - rho[0], a[1] - rho[1], a[2] - rho[2]};
    const double bm[3] = {b[0] - rho[0], b[1] - rho[1], b[2] - rho[2]};
    const double t0 = am[0] * u[0] + am[1] * u[1] + am[2] * u[2];
    const double lp = bm[0] * t[0] + bm[1] * t[1] + bm[2] * t[2];
    const double lm = am[0] * t[0] + am[1] * t[1] + am[2] * t[2];
    const double Rp = sqrt((r[0] - b[0]) * (r[0] - b[0]) + (r[1] - b[1]) * (r[1] - b[1]) + (r[2] - b[2]) * (r[2] - b[2]));
    const double Rm = sqrt((r[0] - a[0]) * (r[0] - a[0]) + (r[1] - a[1]) * (r[1] - a[1]) + (r[2] - a[2]) * (r[2] - a[2]));
    const double R02 = t0 * t0 + d * d;
    double f;
    if (lm >= 0)
      f = log((Rp + lp) / (Rm + lm));
    else if (lp <= 0)
      f = log((Rm - lm) / (Rp - lp));
    else
      f = log((Rp + lp) * (Rm - lm) / R02);
    const double beta = atan2(t0 * lp, R02 + ad * Rp) - atan2(t0 * lm, R02 + ad * Rm);
    const double F1 = 0.5 * (lp * Rp - lm * Rm) + 0.5 * R02 * f;
    const double F3 = 0.25 * (lp * Rp * Rp * Rp - lm * Rm * Rm * Rm) + 0.375 * R02 * (lp * Rp - lm * Rm) +
                      0.375 * R02 * R02 * f;
    sum_t0f += t0 * f;
    sum_beta += beta;
    sum_t0F1 += t0 * F1;
    for (int c = 0; c < 3; ++c) {
      pm1[c] += u[c] * F1;
      p1[c] += u[c] * F3;
      uf[c] += u[c] * f;
    }
  }
  o.Im1 = sum_t0f - ad * sum_beta;
  o.I1 = (d * d * o.Im1 + sum_t0F1) / 3.0;
  const double sg = (d > 0) - (d < 0);
  for (int c = 0; c < 3; ++c) {
    o.Vm1[c] = pm1[c] - d * o.Im1 * n[c];
    o.V1[c] = p1[c] / 3.0 - d * o.I1 * n[c];
    o.Gm3[c] = uf[c] + sg * sum_beta * n[c];
  }
}

// Stage 1: one thread per (near pair, outer point k of P).  Inner integrals
// over Q at r_k: per medium J0 = int G and J1 = int G r' (4 complex each),
// and, unless the pair is coplanar, V = int (g1 + g2)(r - r') (3 complex).
constexpr int NEAR_VALS = 11;

__global__ void __launch_bounds__(64) near_inner_kernel(const double* __restrict__ xyz9, const double* __restrict__ area,
                                                        const NearPair* __restrict__ near, int64_t nnear, FillConsts fc,
                                                        cd* __restrict__ buf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnear * 7) return;
  const int64_t pi = t / 7;
  const int k = (int)(t % 7);
  const NearPair np = near[pi];
  double vp[3][3], vq[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      vp[a][c] = xyz9[(int64_t)np.p * 9 + a * 3 + c];
      vq[a][c] = xyz9[(int64_t)np.q * 9 + a * 3 + c];
    }
  double r[3];
  for (int c = 0; c < 3; ++c) r[c] = fc.bary[k][0] * vp[0][c] + fc.bary[k][1] * vp[1][c] + fc.bary[k][2] * vp[2][c];
  Pot pot;
  tri_potentials(r, vq, pot);
  const double Aq = area[np.q];
  const double i4p = 0.25 / M_PI;
  const double kr[2] = {fc.k1, fc.k2r}, ki[2] = {0.0, fc.k2i};
  cd* o = buf + t * NEAR_VALS;
  for (int m = 0; m < 2; ++m) {
    const double k2r = kr[m] * kr[m] - ki[m] * ki[m], k2i = 2 * kr[m] * ki[m];
    cd J0 = cscale({pot.Im1 - 0.5 * k2r * pot.I1, -0.5 * k2i * pot.I1}, i4p);
    cd J1[3];
    for (int c = 0; c < 3; ++c) {
      const double a0 = pot.Vm1[c] + r[c] * pot.Im1, a1 = pot.V1[c] + r[c] * pot.I1;
      J1[c] = cscale({a0 - 0.5 * k2r * a1, -0.5 * k2i * a1}, i4p);
    }
    for (int l = 0; l < 7; ++l) {
      double rq[3];
      for (int c = 0; c < 3; ++c) rq[c] = fc.bary[l][0] * vq[0][c] + fc.bary[l][1] * vq[1][c] + fc.bary[l][2] * vq[2][c];
      const double R = sqrt((r[0] - rq[0]) * (r[0] - rq[0]) + (r[1] - rq[1]) * (r[1] - rq[1]) + (r[2] - rq[2]) * (r[2] - rq[2]));
      const cd gr = cscale(Gr_rem(kr[m], ki[m], R), Aq * fc.w[l]);
      J0 = cadd(J0, gr);
      for (int c = 0; c < 3; ++c) J1[c] = cadd(J1[c], cscale(gr, rq[c]));
    }
    o[4 * m] = J0;
    for (int c = 0; c < 3; ++c) o[4 * m + 1 + c] = J1[c];
  }
  cd V[3] = {{0, 0}, {0, 0}, {0, 0}};
  if (!np.coplanar) {
    for (int c = 0; c < 3; ++c)
      V[c] = cscale({2.0 * pot.Gm3[c] - 0.5 * fc.ksq_re * pot.Vm1[c], -0.5 * fc.ksq_im * pot.Vm1[c]}, -i4p);
    for (int l = 0; l < 7; ++l) {
      double rq[3];
      for (int c = 0; c < 3; ++c) rq[c] = fc.bary[l][0] * vq[0][c] + fc.bary[l][1] * vq[1][c] + fc.bary[l][2] * vq[2][c];
      const double R = sqrt((r[0] - rq[0]) * (r[0] - rq[0]) + (r[1] - rq[1]) * (r[1] - rq[1]) + (r[2] - rq[2]) * (r[2] - rq[2]));
      const cd g = cadd(gr_rem(kr[0], ki[0], R), gr_rem(kr[1], ki[1], R));
      const cd gw = cscale(g, Aq * fc.w[l]);
      for (int c = 0; c < 3; ++c) V[c] = cadd(V[c], cscale(gw, r[c] - rq[c]));
    }
  }
  for (int c = 0; c < 3; ++c) o[8 + c] = V[c];
}

// Stage 2: one thread per near pair; outer 7-point rule on P:
//   T_i[a,b] = j k_i c_a c_b / A_Q sum_k w_k [ (r_k - p_a).(J1 - q_b J0)/4 - J0 / k_i^2 ]
//   K[a,b]   = -c_a c_b / (4 A_Q) sum_k w_k (r_k - p_a).(V x (r_k - q_b))
template <typename R>
__global__ void __launch_bounds__(64) near_outer_kernel(const double* __restrict__ xyz9, const double* __restrict__ area,
                                                        const double* __restrict__ cl64, int64_t nt,
                                                        const NearPair* __restrict__ near, int64_t nnear, FillConsts fc,
                                                        const cd* __restrict__ buf, cx<R>* __restrict__ out,
                                                        int64_t op_stride, int64_t ldl,
                                                        const NearOut* __restrict__ outs, int cell0, int transposed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnear) return;
  const NearPair np = near[t];
  if (outs) {  // batched: the pair's own block
    const NearOut ob = outs[np.pad - cell0];
    out += ob.off;
    op_stride = ob.op_stride;
    ldl = ob.ldl;
  }
  const int P = np.p, Q = np.q;
  double vp[3][3], vq[3][3], ca[3], cb[3];
  for (int a = 0; a < 3; ++a) {
    ca[a] = cl64[a * nt + P];
    cb[a] = cl64[a * nt + Q];
    for (int c = 0; c < 3; ++c) {
      vp[a][c] = xyz9[(int64_t)P * 9 + a * 3 + c];
      vq[a][c] = xyz9[(int64_t)Q * 9 + a * 3 + c];
    }
  }
  const double Aq = area[Q];
  cd Kab[3][3] = {}, Tab[2][3][3] = {};
  for (int k = 0; k < 7; ++k) {
    const cd* in = buf + (t * 7 + k) * NEAR_VALS;
    double r[3];
    for (int c = 0; c < 3; ++c) r[c] = fc.bary[k][0] * vp[0][c] + fc.bary[k][1] * vp[1][c] + fc.bary[k][2] * vp[2][c];
    const double wk = fc.w[k];
    for (int m = 0; m < 2; ++m) {
      const cd J0 = in[4 * m], J1[3] = {in[4 * m + 1], in[4 * m + 2], in[4 * m + 3]};
      const cd jk = {fc.jk[m][0], fc.jk[m][1]}, ik2 = {fc.ik2[m][0], fc.ik2[m][1]};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          cd sacc = {0, 0};
          for (int c = 0; c < 3; ++c) sacc = cadd(sacc, cscale(csub(J1[c], cscale(J0, vq[b][c])), r[c] - vp[a][c]));
          sacc = csub(cscale(sacc, 0.25), cmul(J0, ik2));
          Tab[m][a][b] = cadd(Tab[m][a][b], cscale(cmul(jk, sacc), wk * ca[a] * cb[b] / Aq));
        }
    }
    if (!np.coplanar) {
      const cd V[3] = {in[8], in[9], in[10]};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          cd sacc = {0, 0};
          for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const cd vx = csub(cscale(V[c1], r[c2] - vq[b][c2]), cscale(V[c2], r[c1] - vq[b][c1]));
            sacc = cadd(sacc, cscale(vx, r[c] - vp[a][c]));
          }
          Kab[a][b] = cadd(Kab[a][b], cscale(sacc, -wk * ca[a] * cb[b] / (4.0 * Aq)));
        }
    }
  }
  // (transposed: the block of test P and source Q goes to the slot of the
  // reversed pair, row i = Q's position, column j = P's, entry (b, a))
  cx<R>* o0 = out + (3 * (int64_t)np.i) * ldl + 3 * (int64_t)np.j;
  const int64_t sa = transposed ? 1 : ldl, sb = transposed ? ldl : 1;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      o0[a * sa + b * sb] = cx<R>{(R)Kab[a][b].re, (R)Kab[a][b].im};
      for (int o = 0; o < 2; ++o) {
        cd v = {0, 0};
        for (int m = 0; m < 2; ++m) v = cadd(v, cmul({fc.e[o][m][0], fc.e[o][m][1]}, Tab[m][a][b]));
        o0[(o + 1) * op_stride + a * sa + b * sb] = cx<R>{(R)v.re, (R)v.im};
      }
    }
}

// Bytes of the near-pair stage's intermediate values for nnear pairs.
size_t near_buffer_bytes(int64_t nnear) { return (size_t)nnear * 7 * NEAR_VALS * sizeof(cd); }

// The two near-pair launches; their intermediate values go to buf_in
// (near_buffer_bytes(nnear) bytes of device memory), or to stream-ordered
// scratch when buf_in is NULL.
template <typename R>
static void near_stage(const cbfm_mesh_s* m, const FillConsts& fc, const NearPair* near, int64_t nnear, cx<R>* out,
                       int64_t op_stride, int64_t ldl, hipStream_t s, const NearOut* outs = nullptr, int cell0 = 0,
                       void* buf_in = nullptr, int transposed = 0) {
  if (nnear == 0) return;
  Scratch own(buf_in ? 0 : near_buffer_bytes(nnear), s);
  cd* buf = static_cast<cd*>(buf_in ? buf_in : own.p);
  hipLaunchKernelGGL(near_inner_kernel, dim3((unsigned)((nnear * 7 + 63) / 64)), dim3(64), 0, s, m->tri_xyz.as<double>(),
                     m->area.as<double>(), near, nnear, fc, buf);
  CBFM_HIP(hipGetLastError());
  hipLaunchKernelGGL((near_outer_kernel<R>), dim3((unsigned)((nnear + 63) / 64)), dim3(64), 0, s, m->tri_xyz.as<double>(),
                     m->area.as<double>(), m->c64.as<double>(), m->h.nt, near, nnear, fc, buf, out, op_stride,
                     ldl, outs, cell0, transposed);
  CBFM_HIP(hipGetLastError());
}

void fill_local(const cbfm_mesh_s* m, const Media& md, int precision, int layout,
                const int32_t* rowTris, int64_t nrt, const int32_t* colTris, int64_t nct,
                const NearPair* near, int64_t nnear, void* local, hipStream_t s, void* near_buf) {
  const FillConsts fc = make_consts(md, layout);
  const int64_t ldl = 3 * nct, op_stride = 3 * nrt * ldl;
  const bool lossy = md.k2i != 0.0;
  CBFM_REQUIRE(nrt <= 65535, CBFM_E_ARG, "too many row triangles for one launch");
  dim3 grid((unsigned)((nct + 255) / 256), (unsigned)nrt);
  {
  TimedLaunch tl(precision == CBFM_FP64 ? T_FILL_REGULAR : T_FILL_REGULAR_F32, s,
                 (double)nrt * (double)nct);  // work: triangle pairs
  if (precision == CBFM_FP64) {
    auto* out = static_cast<cx<double>*>(local);
    if (lossy)
      hipLaunchKernelGGL((fill_regular_kernel<double, true>), grid, dim3(256), 0, s, m->tab64(), rowTris,
                         colTris, nct, fc, out, op_stride, ldl);
    else
      hipLaunchKernelGGL((fill_regular_kernel<double, false>), grid, dim3(256), 0, s, m->tab64(), rowTris,
                         colTris, nct, fc, out, op_stride, ldl);
    CBFM_HIP(hipGetLastError());
  } else {
    auto* out = static_cast<cx<float>*>(local);
    if (lossy)
      hipLaunchKernelGGL((fill_regular_kernel<float, true>), grid, dim3(256), 0, s, m->tab32(), rowTris,
                         colTris, nct, fc, out, op_stride, ldl);
    else
      hipLaunchKernelGGL((fill_regular_kernel<float, false>), grid, dim3(256), 0, s, m->tab32(), rowTris,
                         colTris, nct, fc, out, op_stride, ldl);
  }
  CBFM_HIP(hipGetLastError());
  }
  TimedLaunch tn(T_FILL_NEAR, s, (double)nnear);  // work: near pairs
  if (precision == CBFM_FP64)
    near_stage(m, fc, near, nnear, static_cast<cx<double>*>(local), op_stride, ldl, s, nullptr, 0, near_buf);
  else
    near_stage(m, fc, near, nnear, static_cast<cx<float>*>(local), op_stride, ldl, s, nullptr, 0, near_buf);
}

void fill_near(const cbfm_mesh_s* m, const Media& md, int precision, int layout, const NearPair* near, int64_t nnear,
               int64_t nrt, int64_t nct, void* local, hipStream_t s, int transposed) {
  const FillConsts fc = make_consts(md, layout);
  const int64_t ldl = 3 * nct, op_stride = 3 * nrt * ldl;
  TimedLaunch tn(T_FILL_NEAR, s, (double)nnear);  // work: near pairs
  if (precision == CBFM_FP64)
    near_stage(m, fc, near, nnear, static_cast<cx<double>*>(local), op_stride, ldl, s, nullptr, 0, nullptr, transposed);
  else
    near_stage(m, fc, near, nnear, static_cast<cx<float>*>(local), op_stride, ldl, s, nullptr, 0, nullptr, transposed);
}

void fill_near_batch(const cbfm_mesh_s* m, const Media& md, int layout, const NearPair* near, int64_t nnear,
                     const NearOut* outs, int cell0, void* local, hipStream_t s) {
  const FillConsts fc = make_consts(md, layout);
  TimedLaunch tn(T_FILL_NEAR, s, (double)nnear);  // work: near pairs
  near_stage(m, fc, near, nnear, static_cast<cx<double>*>(local), 0, 0, s, outs, cell0);
}

template <typename R>
static void batch_launch(const std::vector<FillBatchItem>& items, hipStream_t s) {
  std::vector<FillJob<R>> jobs;
  int64_t total = 0;
  double pairs = 0;
  for (const FillBatchItem& it : items) {
    if (it.nrt == 0 || it.nct == 0) continue;
    FillJob<R> j{};
    if constexpr (std::is_same<R, double>::value)
      j.tab = it.m->tab64();
    else
      j.tab = it.m->tab32();
    j.fc = make_consts(it.md, it.layout);
    j.rowTris = it.rowTris;
    j.colTris = it.colTris;
    j.nct = it.nct;
    j.ldl = 3 * it.nct;
    j.op_stride = 3 * it.nrt * j.ldl;
    j.out = static_cast<cx<R>*>(it.local);
    j.lossy = it.md.k2i != 0.0;
    j.item0 = total;
    total += it.nrt * ((it.nct + 255) / 256);
    pairs += (double)it.nrt * (double)it.nct;
    jobs.push_back(j);
  }
  if (jobs.empty()) return;
  Scratch dev(jobs.size() * sizeof(FillJob<R>), s);
  CBFM_HIP(hipMemcpyAsync(dev.p, jobs.data(), jobs.size() * sizeof(FillJob<R>), hipMemcpyHostToDevice, s));
  int dev_id = 0, cus = 0;
  CBFM_HIP(hipGetDevice(&dev_id));
  CBFM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
  const int64_t grid = std::min<int64_t>(total, (int64_t)8 * std::max(cus, 1));
  {
    TimedLaunch tl(std::is_same<R, double>::value ? T_FILL_REGULAR : T_FILL_REGULAR_F32, s,
                   pairs);  // work: triangle pairs
    hipLaunchKernelGGL(fill_regular_batch_kernel<R>, dim3((unsigned)grid), dim3(256), 0, s, dev.as<FillJob<R>>(),
                       (int)jobs.size(), total);
    CBFM_HIP(hipGetLastError());
  }
  CBFM_HIP(hipStreamSynchronize(s));  // the job table is host memory of this frame
}

void fill_regular_batch(const std::vector<FillBatchItem>& items, int precision, hipStream_t s) {
  if (precision == CBFM_FP64)
    batch_launch<double>(items, s);
  else
    batch_launch<float>(items, s);
}

// ------------------------------------------------------------- assembly
// Z[o][r][c] = sum over the two triangles of RWG row0+r and of RWG col0+c of
// the local entries (signs and lengths are inside the local blocks).
template <typename R, typename RO>
__global__ void assemble_kernel(const cx<R>* __restrict__ local, int64_t op_stride, int64_t ldl,
                                const int32_t* __restrict__ rowEdges, int64_t nrow,
                                const int32_t* __restrict__ colEdges, int64_t ncol,
                                const int32_t* __restrict__ tplus, const int32_t* __restrict__ tminus,
                                const int32_t* __restrict__ aplus, const int32_t* __restrict__ aminus,
                                const int32_t* __restrict__ rowPos, const int32_t* __restrict__ colPos,
                                cx<RO>* __restrict__ Z, int64_t zop_stride, int64_t ldz) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= ncol) return;
  const int32_t em = rowEdges[r], en = colEdges[c];
  const int64_t ri[2] = {3 * (int64_t)rowPos[tplus[em]] + aplus[em], 3 * (int64_t)rowPos[tminus[em]] + aminus[em]};
  const int64_t ci[2] = {3 * (int64_t)colPos[tplus[en]] + aplus[en], 3 * (int64_t)colPos[tminus[en]] + aminus[en]};
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    RO re = 0, im = 0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const cx<R> v = local[o * op_stride + ri[x] * ldl + ci[y]];
        re += (RO)v.re;
        im += (RO)v.im;
      }
    Z[o * zop_stride + r * ldz + c] = cx<RO>{re, im};
  }
}

void assemble(const cbfm_mesh_s* m, int precision, const void* local, int64_t nrt, int64_t nct,
              const int32_t* rowEdges, int64_t nrow, const int32_t* colEdges, int64_t ncol,
              const int32_t* rowPos, const int32_t* colPos, void* Z, int64_t zop_stride, int64_t ldz,
              hipStream_t s, int out_fp64) {
  const int64_t ldl = 3 * nct, op_stride = 3 * nrt * ldl;
  CBFM_REQUIRE(nrow <= 65535, CBFM_E_ARG, "too many rows for one assembly launch");
  dim3 grid((unsigned)((ncol + 255) / 256), (unsigned)nrow);
  TimedLaunch tl(T_ASSEMBLE, s);
  const int32_t *tp = m->tplus.as<int32_t>(), *tm = m->tminus.as<int32_t>();
  const int32_t *ap = m->aplus.as<int32_t>(), *am = m->aminus.as<int32_t>();
  if (precision == CBFM_FP64)
    hipLaunchKernelGGL((assemble_kernel<double, double>), grid, dim3(256), 0, s,
                       static_cast<const cx<double>*>(local), op_stride, ldl, rowEdges, nrow, colEdges, ncol, tp, tm,
                       ap, am, rowPos, colPos, static_cast<cx<double>*>(Z), zop_stride, ldz);
  else if (out_fp64)
    hipLaunchKernelGGL((assemble_kernel<float, double>), grid, dim3(256), 0, s, static_cast<const cx<float>*>(local),
                       op_stride, ldl, rowEdges, nrow, colEdges, ncol, tp, tm, ap, am, rowPos, colPos,
                       static_cast<cx<double>*>(Z), zop_stride, ldz);
  else
    hipLaunchKernelGGL((assemble_kernel<float, float>), grid, dim3(256), 0, s, static_cast<const cx<float>*>(local),
                       op_stride, ldl, rowEdges, nrow, colEdges, ncol, tp, tm, ap, am, rowPos, colPos,
                       static_cast<cx<float>*>(Z), zop_stride, ldz);
  CBFM_HIP(hipGetLastError());
}

// The same gather for a list of RWG pairs (pairs[2k] = row r < nrow,
// pairs[2k + 1] = column c < ncol of the listed edges), written to
// Z[op][r][c]: the entries of an assembled block whose triangle-local
// values have since been overwritten in some slots.  The sum runs in the
// order of assemble_kernel, so an entry whose slots did not change is
// reproduced bit for bit.
template <typename R, typename RO>
__global__ void assemble_pairs_kernel(const cx<R>* __restrict__ local, int64_t op_stride, int64_t ldl,
                                      const int32_t* __restrict__ rowEdges, const int32_t* __restrict__ colEdges,
                                      const int32_t* __restrict__ pairs, int64_t npairs,
                                      const int32_t* __restrict__ tplus, const int32_t* __restrict__ tminus,
                                      const int32_t* __restrict__ aplus, const int32_t* __restrict__ aminus,
                                      const int32_t* __restrict__ rowPos, const int32_t* __restrict__ colPos,
                                      cx<RO>* __restrict__ Z, int64_t zop_stride, int64_t ldz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npairs) return;
  const int64_t r = pairs[2 * k], c = pairs[2 * k + 1];
  const int32_t em = rowEdges[r], en = colEdges[c];
  const int64_t ri[2] = {3 * (int64_t)rowPos[tplus[em]] + aplus[em], 3 * (int64_t)rowPos[tminus[em]] + aminus[em]};
  const int64_t ci[2] = {3 * (int64_t)colPos[tplus[en]] + aplus[en], 3 * (int64_t)colPos[tminus[en]] + aminus[en]};
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    RO re = 0, im = 0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const cx<R> v = local[o * op_stride + ri[x] * ldl + ci[y]];
        re += (RO)v.re;
        im += (RO)v.im;
      }
    Z[o * zop_stride + r * ldz + c] = cx<RO>{re, im};
  }
}

void assemble_pairs(const cbfm_mesh_s* m, int precision, const void* local, int64_t nrt, int64_t nct,
                    const int32_t* rowEdges, const int32_t* colEdges, const int32_t* pairs, int64_t npairs,
                    const int32_t* rowPos, const int32_t* colPos, void* Z, int64_t zop_stride, int64_t ldz,
                    hipStream_t s, int out_fp64) {
  if (npairs == 0) return;
  const int64_t ldl = 3 * nct, op_stride = 3 * nrt * ldl;
  const dim3 grid((unsigned)((npairs + 255) / 256));
  TimedLaunch tl(T_ASSEMBLE, s);
  const int32_t *tp = m->tplus.as<int32_t>(), *tm = m->tminus.as<int32_t>();
  const int32_t *ap = m->aplus.as<int32_t>(), *am = m->aminus.as<int32_t>();
  if (precision == CBFM_FP64)
    hipLaunchKernelGGL((assemble_pairs_kernel<double, double>), grid, dim3(256), 0, s,
                       static_cast<const cx<double>*>(local), op_stride, ldl, rowEdges, colEdges, pairs, npairs, tp,
                       tm, ap, am, rowPos, colPos, static_cast<cx<double>*>(Z), zop_stride, ldz);
  else if (out_fp64)
    hipLaunchKernelGGL((assemble_pairs_kernel<float, double>), grid, dim3(256), 0, s,
                       static_cast<const cx<float>*>(local), op_stride, ldl, rowEdges, colEdges, pairs, npairs, tp, tm,
                       ap, am, rowPos, colPos, static_cast<cx<double>*>(Z), zop_stride, ldz);
  else
    hipLaunchKernelGGL((assemble_pairs_kernel<float, float>), grid, dim3(256), 0, s,
                       static_cast<const cx<float>*>(local), op_stride, ldl, rowEdges, colEdges, pairs, npairs, tp, tm,
                       ap, am, rowPos, colPos, static_cast<cx<float>*>(Z), zop_stride, ldz);
  CBFM_HIP(hipGetLastError());
}

// ------------------------------------------------------------- RHS
__global__ void rhs_kernel(const double* __restrict__ xyz9, const int32_t* __restrict__ tplus,
                           const int32_t* __restrict__ tminus, const int32_t* __restrict__ aplus,
                           const int32_t* __restrict__ aminus, const double* __restrict__ length,
                           int64_t ne, const double* __restrict__ inc, int64_t nrhs, FillConsts fc,
                           double eta0, cd* __restrict__ v) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (m >= ne) return;
  const double kh[3] = {inc[c * 6 + 0], inc[c * 6 + 1], inc[c * 6 + 2]};
  const double ph[3] = {inc[c * 6 + 3], inc[c * 6 + 4], inc[c * 6 + 5]};
  // H direction k x p
  const double hh[3] = {kh[1] * ph[2] - kh[2] * ph[1], kh[2] * ph[0] - kh[0] * ph[2], kh[0] * ph[1] - kh[1] * ph[0]};
  cd vE = {0, 0}, vH = {0, 0};
  for (int side = 0; side < 2; ++side) {
    const int t = side ? tminus[m] : tplus[m];
    const int a = side ? aminus[m] : aplus[m];
    const double sgn = side ? -1.0 : 1.0;
    const double* P = xyz9 + (int64_t)t * 9;
    for (int k = 0; k < 7; ++k) {
      double r[3];
      for (int x = 0; x < 3; ++x) r[x] = fc.bary[k][0] * P[x] + fc.bary[k][1] * P[3 + x] + fc.bary[k][2] * P[6 + x];
      // int f . E = sum_k w_k A (s l / 2A)(r - p) . E = sum_k w_k (s l / 2)(r - p) . E
      double dE = 0, dH = 0;
      for (int x = 0; x < 3; ++x) {
        dE += (r[x] - P[a * 3 + x]) * ph[x];
        dH += (r[x] - P[a * 3 + x]) * hh[x];
      }
      const double kr = kh[0] * r[0] + kh[1] * r[1] + kh[2] * r[2];
      double sn, cs;
      sincos(fc.k1 * kr, &sn, &cs);  // e^{-j k0 k.r} = cs - j sn
      const double f = fc.w[k] * sgn * length[m] * 0.5;
      vE.re += f * dE * cs;
      vE.im -= f * dE * sn;
      vH.re -= f * dH * cs / eta0;
      vH.im += f * dH * sn / eta0;
    }
  }
  v[c * 2 * ne + m] = vE;
  v[c * 2 * ne + ne + m] = vH;
}

void rhs_launch(const cbfm_mesh_s* m, const Media& md, double eta0, const double* inc_dev, int64_t nrhs,
                void* v_dev, hipStream_t s) {
  const FillConsts fc = make_consts(md, CBFM_LAYOUT_OPS3);
  dim3 grid((unsigned)((m->h.ne + 255) / 256), (unsigned)nrhs);
  hipLaunchKernelGGL(rhs_kernel, grid, dim3(256), 0, s, m->tri_xyz.as<double>(), m->tplus.as<int32_t>(),
                     m->tminus.as<int32_t>(), m->aplus.as<int32_t>(), m->aminus.as<int32_t>(),
                     m->length.as<double>(), m->h.ne, inc_dev, nrhs, fc, eta0, static_cast<cd*>(v_dev));
  CBFM_HIP(hipGetLastError());
}

}  // namespace cbfm

using namespace cbfm;

namespace cbfm {

// The fill of RWG rows row0..row0+nrow-1 against columns col0..col0+ncol-1
// into out (3 matrices, ld), after the arguments are checked.  Its device
// workspace (index tables, near-pair intermediates, triangle-local blocks,
// each 256-byte aligned) is carved from ws (ws_bytes long) when given, else
// taken from stream-ordered scratch.  Synchronises s (host staging).
static void fill_ranges(const cbfm_mesh_s* m, const Media& md, int precision, int64_t row0, int64_t nrow, int64_t col0,
                        int64_t ncol, int layout, void* out_dev, int64_t ld, hipStream_t s, char* ws, size_t ws_bytes) {
  const MeshHost& h = m->h;
  // triangles touching the ranges and their positions
  auto tris_of = [&](int64_t e0, int64_t n, std::vector<int32_t>& list, std::vector<int32_t>& pos) {
    pos.assign(h.nt, -1);
    for (int64_t e = e0; e < e0 + n; ++e) {
      pos[h.tplus[e]] = 0;
      pos[h.tminus[e]] = 0;
    }
    list.clear();
    for (int64_t t = 0; t < h.nt; ++t)
      if (pos[t] == 0) {
        pos[t] = (int32_t)list.size();
        list.push_back((int32_t)t);
      }
  };
  std::vector<int32_t> rl, rp, cl, cp;
  tris_of(row0, nrow, rl, rp);
  tris_of(col0, ncol, cl, cp);
  std::vector<NearPair> nl;
  for (const NearPair& q : h.near)
    if (rp[q.p] >= 0 && cp[q.q] >= 0) nl.push_back({q.p, q.q, rp[q.p], cp[q.q], q.coplanar, 0});
  std::vector<int32_t> re(nrow), ce(ncol);
  for (int64_t r = 0; r < nrow; ++r) re[r] = (int32_t)(row0 + r);
  for (int64_t c = 0; c < ncol; ++c) ce[c] = (int32_t)(col0 + c);
  const int64_t nrt = rl.size(), nct = cl.size();
  const size_t esz = precision == CBFM_FP64 ? 16 : 8;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t ib = sizeof(int32_t) * (rl.size() + cl.size() + rp.size() + cp.size() + re.size() + ce.size()) +
                    sizeof(NearPair) * nl.size();
  const size_t nb = near_buffer_bytes((int64_t)nl.size()), lb = 3 * 9 * (size_t)nrt * nct * esz;
  const size_t total = al(ib) + al(nb) + al(lb);
  std::unique_ptr<Scratch> own;
  if (ws) {
    CBFM_REQUIRE(total <= ws_bytes, CBFM_E_ARG,
                 "the fill of these ranges needs " + std::to_string(total) + " bytes of workspace; the maximum is " +
                     std::to_string(ws_bytes));
  } else {
    own.reset(new Scratch(total, s));
    ws = own->as<char>();
  }
  char* p = ws;
  std::vector<char> host(ib);
  size_t off = 0;
  auto put = [&](const void* src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + off, src, bytes);
    void* dst = p + off;
    off += bytes;
    return dst;
  };
  auto* d_rl = (int32_t*)put(rl.data(), rl.size() * 4);
  auto* d_cl = (int32_t*)put(cl.data(), cl.size() * 4);
  auto* d_rp = (int32_t*)put(rp.data(), rp.size() * 4);
  auto* d_cp = (int32_t*)put(cp.data(), cp.size() * 4);
  auto* d_re = (int32_t*)put(re.data(), re.size() * 4);
  auto* d_ce = (int32_t*)put(ce.data(), ce.size() * 4);
  auto* d_nl = (NearPair*)put(nl.data(), nl.size() * sizeof(NearPair));
  CBFM_HIP(hipMemcpyAsync(p, host.data(), ib, hipMemcpyHostToDevice, s));
  void* near_buf = ws + al(ib);
  void* local = ws + al(ib) + al(nb);
  fill_local(m, md, precision, layout, d_rl, nrt, d_cl, nct, d_nl, (int64_t)nl.size(), local, s, near_buf);
  assemble(m, precision, local, nrt, nct, d_re, nrow, d_ce, ncol, d_rp, d_cp, out_dev, nrow * ld, ld, s);
  // the host staging buffer must outlive the asynchronous copy
  CBFM_HIP(hipStreamSynchronize(s));
}

// K1 = Kv / 2 and K2 = K - K1 (Kv: the K operator of a body whose interior
// medium is the exterior one, which is 2 K1 bit for bit)
template <typename R>
__global__ void split_k_kernel(const cx<R>* __restrict__ Kv, cx<R>* __restrict__ K1, cx<R>* __restrict__ K2, int64_t ncol,
                               int64_t ld) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= ncol) return;
  const cx<R> v = Kv[r * ld + c], k = K2[r * ld + c];
  const cx<R> k1 = {v.re * (R)0.5, v.im * (R)0.5};
  K1[r * ld + c] = k1;
  K2[r * ld + c] = cx<R>{k.re - k1.re, k.im - k1.im};
}

static void fill_check(cbfm_mesh m, int32_t precision, int64_t row0, int64_t nrow, int64_t col0, int64_t ncol,
                       int32_t layout, const void* out_dev, int64_t ld) {
  CBFM_REQUIRE(m != nullptr && out_dev != nullptr, CBFM_E_ARG, "mesh or output is NULL");
  CBFM_REQUIRE(precision == CBFM_FP64 || precision == CBFM_FP32, CBFM_E_ARG, "unknown precision");
  CBFM_REQUIRE(layout == CBFM_LAYOUT_MEDIA3 || layout == CBFM_LAYOUT_OPS3 || layout == CBFM_LAYOUT_MEDIA4, CBFM_E_ARG,
               "unknown layout");
  const MeshHost& h = m->h;
  CBFM_REQUIRE(row0 >= 0 && nrow >= 0 && row0 + nrow <= h.ne && col0 >= 0 && ncol >= 0 && col0 + ncol <= h.ne,
               CBFM_E_ARG, "row/column range outside [0, ne)");
  CBFM_REQUIRE(ld >= ncol, CBFM_E_ARG, "ld < ncol");
}

// ------------------------------------------------------------- allocation-free fill
// Workspace of cbfm_fill_pmchwt_noalloc: one array per device, held until
// the process ends.  Host code never uses the array's name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = (size_t)CBFM_FILL_NOALLOC_MAX_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static char* noalloc_scratch() {
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  CBFM_REQUIRE(dev >= 0 && dev < kMaxDevices, CBFM_E_ARG, "device index above the workspace table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    CBFM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    CBFM_REQUIRE(ptr != nullptr, CBFM_E_HIP, "no device address for the fill workspace");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

}  // namespace cbfm

extern "C" cbfm_status cbfm_fill_pmchwt(cbfm_mesh m, const cbfm_medium* med, int32_t precision, int64_t row0,
                                        int64_t nrow, int64_t col0, int64_t ncol, int32_t layout, void* out_dev,
                                        int64_t ld, void* stream) {
  return guarded([&] {
    fill_check(m, precision, row0, nrow, col0, ncol, layout, out_dev, ld);
    const Media md = make_media(med);
    if (nrow == 0 || ncol == 0) return;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (layout != CBFM_LAYOUT_MEDIA4) {
      fill_ranges(m, md, precision, row0, nrow, col0, ncol, layout, out_dev, ld, s, nullptr, 0);
      return;
    }
    // [K1, K2, T1, T2]: [K1 + K2, T1, T2] of the medium into matrices 1..3,
    // then K of the body with the exterior medium inside (2 K1) apart
    const size_t esz = precision == CBFM_FP64 ? 16 : 8, mat = (size_t)nrow * ld * esz;
    char* o = static_cast<char*>(out_dev);
    fill_ranges(m, md, precision, row0, nrow, col0, ncol, CBFM_LAYOUT_MEDIA3, o + mat, ld, s, nullptr, 0);
    cbfm_medium outside = *med;
    outside.eps_re = 1.0;
    outside.eps_im = 0.0;
    outside.mu_re = 1.0;
    outside.mu_im = 0.0;
    Scratch kv(3 * mat, s);
    fill_ranges(m, make_media(&outside), precision, row0, nrow, col0, ncol, CBFM_LAYOUT_MEDIA3, kv.p, ld, s, nullptr,
                0);
    CBFM_REQUIRE(nrow <= 65535, CBFM_E_ARG, "too many rows for one launch");
    const dim3 g((unsigned)((ncol + 255) / 256), (unsigned)nrow);
    if (precision == CBFM_FP64)
      hipLaunchKernelGGL(split_k_kernel<double>, g, dim3(256), 0, s, kv.as<cx<double>>(), (cx<double>*)o,
                         (cx<double>*)(o + mat), ncol, ld);
    else
      hipLaunchKernelGGL(split_k_kernel<float>, g, dim3(256), 0, s, kv.as<cx<float>>(), (cx<float>*)o,
                         (cx<float>*)(o + mat), ncol, ld);
    CBFM_HIP(hipGetLastError());
    CBFM_HIP(hipStreamSynchronize(s));
  });
}

extern "C" cbfm_status cbfm_fill_pmchwt_noalloc(cbfm_mesh m, const cbfm_medium* med, int32_t precision, int64_t row0,
                                                int64_t nrow, int64_t col0, int64_t ncol, int32_t layout,
                                                void* out_dev, int64_t ld, void* stream) {
  return guarded([&] {
    fill_check(m, precision, row0, nrow, col0, ncol, layout, out_dev, ld);
    CBFM_REQUIRE(layout != CBFM_LAYOUT_MEDIA4, CBFM_E_ARG, "the allocation-free fill has no MEDIA4 layout");
    const Media md = make_media(med);
    if (nrow == 0 || ncol == 0) return;
    char* ws = noalloc_scratch();
    fill_ranges(m, md, precision, row0, nrow, col0, ncol, layout, out_dev, ld, static_cast<hipStream_t>(stream), ws,
                kNoAllocBytes);
  });
}

extern "C" cbfm_status cbfm_rhs(cbfm_mesh m, const cbfm_medium* med, const double* inc_host, int64_t nrhs,
                                void* v_dev, void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(m != nullptr && inc_host != nullptr && v_dev != nullptr, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(nrhs >= 0 && nrhs < 65536, CBFM_E_ARG, "nrhs out of range");
    const Media md = make_media(med);
    if (nrhs == 0) return;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Scratch inc(nrhs * 6 * sizeof(double), s);
    CBFM_HIP(hipMemcpyAsync(inc.p, inc_host, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, s));
    rhs_launch(m, md, med->eta0, inc.as<double>(), nrhs, v_dev, s);
    CBFM_HIP(hipStreamSynchronize(s));
  });
}
