// Blocked Gauss-Jordan elimination with tournament pivoting for batches of
// dense complex double matrices.
//
// The CBF build solves every cell's isolated system Z_mm J_m = V_m for all
// generating waves (Sec. III-A), and the CMP needs the inverse of
// B = (C^M)^H G C^J (Sec. III-C).  Both run here as Gauss-Jordan elimination
// over panels of 32 columns.  Each panel step is a few launches on the
// stream, with no host round trip until the end:
//  1. pivot rows: the panel's rows are split into groups of 256, one row per
//     thread held in registers.  Each group runs an LU factorisation of its
//     rows with partial pivoting (largest |re| + |im|, lowest row on ties)
//     and keeps the 32 rows it pivoted on; the rows kept by eight groups make
//     a group of the next round, until one group is left (tournament
//     pivoting).  The last group inverts the 32 x 32 pivot block D
//     (Gauss-Jordan in LDS, in the order the pivots were chosen) and sets
//     the row permutation of the step: the panel's rows K take the pivot
//     rows, and the rows of K that were not chosen take the places the
//     chosen rows outside K leave (paired in order, by wave ballots).  It
//     saves every row's panel entries (after the permutation) for the
//     update;
//  2. row block: over chunks of 64 columns, the permutation is applied and
//     the pivot rows R become D^{-1} R;
//  3. update: every other row i loses A[i, panel] D^{-1} R, one batched
//     matrix-core GEMM with k = 32 (gemm.hip).
// An inversion runs in place: the columns of the inverse take the places of
// the eliminated columns.  The column of the inverse that belongs to row j
// of the input ends up where the permutations took that row, so a last
// gather, driven by the map of which input row each position holds, puts
// the columns in order.  A solve runs on the augmented [Z | V] and
// only updates the columns right of the panel.
#include <algorithm>
#include <string>
#include <vector>

#include "gemm.h"
#include "gj.h"
#include "internal.h"

namespace cbfm {

namespace {

constexpr int kW = 32;          // panel width
constexpr int kGroup = 256;     // rows per pivot group, one per thread
constexpr int kChunk = 64;      // columns per block of the row-block kernel
constexpr int kSwapInts = 128;  // per matrix: pivot rows [0, 32), displaced
                                // positions [32, 64), their sources [64, 96), count [96]

__device__ inline double gj_cabs1(double2 z) { return fabs(z.x) + fabs(z.y); }
__device__ inline double2 gj_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 gj_recip(double2 p) {
  const double d = p.x * p.x + p.y * p.y;
  return make_double2(p.x / d, -p.y / d);
}
// Pivot key of a row: |re| + |im| rounded to float (a positive value stays
// positive) in the high word, the complement of the thread in the low word,
// so that the largest key is the largest entry and, among equals, the lowest
// thread; 0 for a thread without a candidate row.
__device__ inline uint64_t gj_key(bool alive, double2 z, int t) {
  if (!alive) return 0;
  const double m = gj_cabs1(z);
  uint32_t hi = 0;
  if (m > 0.0) hi = __float_as_uint((float)m) | 1u;  // (NaN counts as zero)
  return ((uint64_t)hi << 32) | (uint32_t)~t;
}

struct SelectArgs {
  const double2* A;
  int64_t strideA, ld;
  int n, k, w;
  const int32_t* cand_in;  // candidate rows of this tournament stage (null: the rows k .. n - 1)
  int cand_len;            // entries of cand_in per matrix (-1 marks an empty slot)
  int nsel_groups;         // blocks that select; at the first round the blocks
                           // after them copy the panel entries of rows 0 .. k - 1
  int32_t* cand_out;       // kW slots per group
  int64_t cand_stride;     // entries per matrix of cand_in / cand_out
  int final_round;
  double2* Pcol;   // n x kW per matrix: the panel entries of every row
  double2* Dinv;   // kW x kW per matrix
  int32_t* swaps;  // kSwapInts per matrix
  int32_t* rowat;  // n per matrix: the input row each position holds (null: not kept)
  int32_t* info;   // per matrix: 1 + the first column without a nonzero pivot
};

__global__ void __launch_bounds__(kGroup) gj_select_kernel(SelectArgs p) {
  const int b = blockIdx.y, g = blockIdx.x, t = threadIdx.x;
  const double2* Ab = p.A + (int64_t)b * p.strideA;
  double2* Pc = p.Pcol + (int64_t)b * p.n * kW;
  const int k = p.k, w = p.w;
  if (p.cand_in == nullptr && g >= p.nsel_groups) {
    // (every load is issued before the first store: a load-store chain per
    // entry would wait on memory 32 times in a row)
    const int r = (g - p.nsel_groups) * kGroup + t;
    if (r < k) {
      double2 v[kW];
#pragma unroll
      for (int j = 0; j < kW; ++j) v[j] = j < w ? Ab[(int64_t)r * p.ld + k + j] : make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < kW; ++j)
        if (j < w) Pc[(int64_t)r * kW + j] = v[j];
    }
    return;
  }
  int row = -1;
  if (p.cand_in == nullptr) {
    const int r = k + g * kGroup + t;
    if (r < p.n) row = r;
  } else {
    const int e = g * kGroup + t;
    if (e < p.cand_len) row = p.cand_in[(int64_t)b * p.cand_stride + e];
  }
  double2 a[kW];
#pragma unroll
  for (int j = 0; j < kW; ++j) a[j] = make_double2(0.0, 0.0);
  if (row >= 0) {
#pragma unroll
    for (int j = 0; j < kW; ++j)
      if (j < w) a[j] = Ab[(int64_t)row * p.ld + k + j];
    if (p.cand_in == nullptr) {
#pragma unroll
      for (int j = 0; j < kW; ++j)
        if (j < w) Pc[(int64_t)row * kW + j] = a[j];
    }
  }
  __shared__ uint64_t s_key[kGroup / 64];
  __shared__ double2 s_prow[kW];
  __shared__ int s_sel[kW];
  bool alive = row >= 0;
  int nsel = 0;
  const int lane = t & 63, wave = t >> 6;
  // LU with partial pivoting over the group's rows; column c picks row s_sel[c]
#pragma unroll
  for (int c = 0; c < kW; ++c) {
    if (c < w && nsel == c) {  // (uniform: stops at the first column with no row left)
      uint64_t key = gj_key(alive, a[c], t);
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(key, off, 64);
        key = o > key ? o : key;
      }
      if (lane == 0) s_key[wave] = key;
      __syncthreads();
      uint64_t best = s_key[0];
      for (int q = 1; q < kGroup / 64; ++q) best = s_key[q] > best ? s_key[q] : best;
      const int bw = (int)~(uint32_t)best;
      const bool nonzero = (best >> 32) != 0;
      if (best != 0) {
        if (t == bw) {
#pragma unroll
          for (int j = c; j < kW; ++j) s_prow[j] = a[j];
          s_sel[c] = row;
          alive = false;
        }
        __syncthreads();
        nsel = c + 1;
        if (nonzero) {
          if (alive) {
            const double2 l = gj_mul(a[c], gj_recip(s_prow[c]));
#pragma unroll
            for (int j = c + 1; j < kW; ++j) {
              const double2 x = s_prow[j];
              a[j].x -= l.x * x.x - l.y * x.y;
              a[j].y -= l.x * x.y + l.y * x.x;
            }
          }
        } else if (p.final_round && t == 0 && p.info[b] == 0) {
          p.info[b] = k + c + 1;
        }
      }
    }
  }
  if (!p.final_round) {
    if (t < kW) p.cand_out[(int64_t)b * p.cand_stride + (int64_t)g * kW + t] = t < nsel ? s_sel[t] : -1;
    return;
  }
  if (nsel < w && t == 0 && p.info[b] == 0) p.info[b] = k + nsel + 1;
  // D (the pivot rows' panel entries, identity-padded) and I, then
  // Gauss-Jordan without further interchanges: [D | I] -> [I | D^{-1}]
  __shared__ double2 s_m[kW][2 * kW + 1];
  for (int e = t; e < kW * 2 * kW; e += kGroup) {
    const int i = e / (2 * kW), j = e % (2 * kW);
    double2 v = make_double2(0.0, 0.0);
    if (j < kW) {
      if (i < nsel && j < w)
        v = Ab[(int64_t)s_sel[i] * p.ld + k + j];
      else if (i == j && i >= w)
        v = make_double2(1.0, 0.0);
    } else if (j - kW == i) {
      v = make_double2(1.0, 0.0);
    }
    s_m[i][j] = v;
  }
  const int mi = t >> 3, mq = t & 7;  // this thread: row mi, columns mq + 8 u
  for (int c = 0; c < kW; ++c) {
    __syncthreads();
    const double2 rp = gj_recip(s_m[c][c]);
    const double2 f = s_m[mi][c];
    double2 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = gj_mul(s_m[c][mq + 8 * u], rp);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double2& y = s_m[mi][mq + 8 * u];
      if (mi == c) {
        y = x[u];
      } else {
        y.x -= f.x * x[u].x - f.y * x[u].y;
        y.y -= f.x * x[u].y + f.y * x[u].x;
      }
    }
  }
  __syncthreads();
  double2* Db = p.Dinv + (int64_t)b * kW * kW;
  for (int e = t; e < kW * kW; e += kGroup) Db[e] = s_m[e / kW][kW + e % kW];
  // the permutation: position k + i takes row s_row[i]; the rows of K that
  // were not chosen take the positions s_dd[] that chosen rows outside K
  // leave (s_ds[]: where each comes from)
  __shared__ int s_row[kW], s_dd[kW], s_ds[kW];
  __shared__ int s_nd;
  int32_t* sw = p.swaps + (int64_t)b * kSwapInts;
  if (t < 64) {
    const int i = t;
    const int r = i < w ? (i < nsel ? s_sel[i] : k + i) : 0;
    bool picked = false;
    for (int j = 0; j < nsel; ++j) picked |= s_sel[j] == k + i;
    const bool hole = i < w && r >= k + w, unsel = i < w && !picked;
    const uint64_t hm = __ballot(hole), um = __ballot(unsel), below = (1ull << i) - 1;
    if (hole) s_dd[__popcll(hm & below)] = r;
    if (unsel) s_ds[__popcll(um & below)] = k + i;
    if (i < w) {
      s_row[i] = r;
      sw[i] = r;
    }
    if (i == 0) s_nd = min(__popcll(hm), __popcll(um));
  }
  __syncthreads();
  const int nd = s_nd;
  if (t < nd) {
    sw[kW + t] = s_dd[t];
    sw[2 * kW + t] = s_ds[t];
  }
  if (t == 0) sw[3 * kW] = nd;
  if (p.rowat) {  // (every read before any write)
    int32_t* ra = p.rowat + (int64_t)b * p.n;
    const int v1 = t < w ? ra[s_row[t]] : 0, v2 = t < nd ? ra[s_ds[t]] : 0;
    __syncthreads();
    if (t < w) ra[k + t] = v1;
    if (t < nd) ra[s_dd[t]] = v2;
  }
  // panel entries of the displaced positions: the rows that now sit there
  constexpr int kDU = kW * kW / kGroup;
  double2 dv[kDU];
#pragma unroll
  for (int u = 0; u < kDU; ++u) {
    const int e = t + kGroup * u, d = e / kW, j = e % kW;
    dv[u] = d < nd && j < w ? Ab[(int64_t)s_ds[d] * p.ld + k + j] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int u = 0; u < kDU; ++u) {
    const int e = t + kGroup * u, d = e / kW, j = e % kW;
    if (d < nd && j < w) Pc[(int64_t)s_dd[d] * kW + j] = dv[u];
  }
}

struct RowsArgs {
  double2* A;
  int64_t strideA, ld;
  int ncols, k, w, col0;
  const double2* Dinv;
  const int32_t* swaps;
};

// Columns col0 + 64 blockIdx.x + (0 .. 63) of matrix blockIdx.y: rows K
// (k .. k + w - 1) receive the pivot rows, the displaced positions receive
// the rows of K they held, and rows K become D^{-1} times themselves.  The
// panel's own columns (present only for an inversion) get D^{-1}; their
// other rows are written by the update.
__global__ void __launch_bounds__(256) gj_rows_kernel(RowsArgs p) {
  const int b = blockIdx.y, t = threadIdx.x;
  double2* Ab = p.A + (int64_t)b * p.strideA;
  const int j0 = p.col0 + (int)blockIdx.x * kChunk;
  const int k = p.k, w = p.w;
  __shared__ double2 s_d[kW][kW + 1];
  __shared__ double2 s_r[kW][kChunk];
  __shared__ int s_sw[kSwapInts];
  const int32_t* sw = p.swaps + (int64_t)b * kSwapInts;
  for (int e = t; e <= 3 * kW; e += 256) s_sw[e] = sw[e];
  for (int e = t; e < kW * kW; e += 256) s_d[e / kW][e % kW] = p.Dinv[(int64_t)b * kW * kW + e];
  __syncthreads();
  const int nd = s_sw[3 * kW];
  auto inpanel = [&](int j) { return j >= k && j < k + w; };
  for (int e = t; e < kW * kChunk; e += 256) {
    const int i = e / kChunk, jj = e % kChunk, j = j0 + jj;
    double2 v = make_double2(0.0, 0.0);
    if (i < w && j < p.ncols && !inpanel(j)) v = Ab[(int64_t)s_sw[i] * p.ld + j];
    s_r[i][jj] = v;
  }
  constexpr int kU = kW * kChunk / 256;
  double2 xd[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int e = t + 256 * u, d = e / kChunk, j = j0 + e % kChunk;
    xd[u] = (d < nd && j < p.ncols && !inpanel(j)) ? Ab[(int64_t)s_sw[2 * kW + d] * p.ld + j]
                                                   : make_double2(0.0, 0.0);
  }
  __syncthreads();  // every read of this block's columns is done
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int e = t + 256 * u, d = e / kChunk, j = j0 + e % kChunk;
    if (d < nd && j < p.ncols && !inpanel(j)) Ab[(int64_t)s_sw[kW + d] * p.ld + j] = xd[u];
  }
  const int jj = t & (kChunk - 1), r0 = (t / kChunk) * 8, j = j0 + jj;
  if (j >= p.ncols) return;
  if (inpanel(j)) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (r0 + q < w) Ab[(int64_t)(k + r0 + q) * p.ld + j] = s_d[r0 + q][j - k];
    return;
  }
  double2 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int c = 0; c < w; ++c) {
    const double2 x = s_r[c][jj];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 d = s_d[r0 + q][c];
      acc[q].x += d.x * x.x - d.y * x.y;
      acc[q].y += d.x * x.y + d.y * x.x;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (r0 + q < w) Ab[(int64_t)(k + r0 + q) * p.ld + j] = acc[q];
}

__global__ void gj_iota_kernel(int32_t* __restrict__ x, int n, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < total) x[e] = (int32_t)(e % n);
}

// out_b[i][j] = in_b[i][src_b[j]] (n x n row-major, b = blockIdx.z).
__global__ void gj_gather_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                 const int32_t* __restrict__ src, int n, int64_t strideA) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
  if (j >= n) return;
  const int64_t row = (int64_t)b * strideA + (int64_t)i * n;
  out[row + j] = in[row + src[(int64_t)b * n + j]];
}

// src_b[rowat_b[q]] = q: the position that holds each input row.
__global__ void gj_src_kernel(const int32_t* __restrict__ rowat, int32_t* __restrict__ src, int n, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t b = e / n;
  src[b * n + rowat[e]] = (int32_t)(e - b * n);
}

// The elimination, enqueued on s with no host wait: info_dev (nmat entries)
// receives 0 or 1 + the first column without a nonzero pivot.  An inversion
// ends with the column gather.  Every scratch buffer is released in stream
// order.
void eliminate(double2* A, int64_t strideA, int64_t ld, int n, int ncols, int nmat, bool inverse, int32_t* info_dev,
               hipStream_t s) {
  CBFM_REQUIRE(n >= 1 && n <= 65535 && nmat >= 1 && nmat <= 65535, CBFM_E_ARG,
               "Gauss-Jordan: order in [1, 65535] and at most 65535 matrices");
  CBFM_REQUIRE(ncols >= n && ld >= ncols && strideA >= (int64_t)(n - 1) * ld + ncols, CBFM_E_ARG,
               "Gauss-Jordan: inconsistent matrix layout");
  const int steps = (n + kW - 1) / kW;
  const int gmax = (n + kGroup - 1) / kGroup;
  const int64_t cstride = (int64_t)gmax * kW;
  Scratch pcol((size_t)nmat * n * kW * sizeof(double2), s), dinv((size_t)nmat * kW * kW * sizeof(double2), s),
      swaps((size_t)nmat * kSwapInts * sizeof(int32_t), s),
      rowat(inverse ? (size_t)nmat * n * sizeof(int32_t) : 0, s),
      cand0((size_t)nmat * cstride * sizeof(int32_t), s),
      cand1((size_t)nmat * cstride * sizeof(int32_t), s);
  CBFM_HIP(hipMemsetAsync(info_dev, 0, (size_t)nmat * sizeof(int32_t), s));
  if (inverse) {
    const int64_t total = (int64_t)nmat * n;
    hipLaunchKernelGGL(gj_iota_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rowat.as<int32_t>(), n,
                       total);
    CBFM_HIP(hipGetLastError());
  }
  // the update of every step: rows outside the panel, columns right of it
  // (an inversion: every column; the panel's own columns are overwritten)
  std::vector<std::vector<GemmDesc>> groups(steps);
  for (int st = 0; st < steps; ++st) {
    const int k = st * kW, w = std::min(kW, n - k);
    for (int b = 0; b < nmat; ++b) {
      double2* Ab = A + (int64_t)b * strideA;
      const double2* P = pcol.as<double2>() + (int64_t)b * n * kW;
      const int rr[2][2] = {{0, k}, {k + w, n}};
      for (const auto& r : rr) {
        if (r[1] <= r[0]) continue;
        auto add = [&](int c0, int c1, int acc) {
          if (c1 <= c0) return;
          groups[st].push_back(gemm(P + (int64_t)r[0] * kW, kW, OP_N, Ab + (int64_t)k * ld + c0, ld, OP_N,
                                    Ab + (int64_t)r[0] * ld + c0, ld, r[1] - r[0], c1 - c0, w, -1.0, acc));
        };
        if (inverse) {
          add(0, k, 1);
          add(k + w, n, 1);
          add(k, k + w, 0);
        } else {
          add(k + w, ncols, 1);
        }
      }
    }
  }
  GemmPlan plan(groups, s, false);
  Scratch* cand[2] = {&cand0, &cand1};
  for (int st = 0; st < steps; ++st) {
    const int k = st * kW, w = std::min(kW, n - k);
    SelectArgs a{};
    a.A = A;
    a.strideA = strideA;
    a.ld = ld;
    a.n = n;
    a.k = k;
    a.w = w;
    a.cand_stride = cstride;
    a.Pcol = pcol.as<double2>();
    a.Dinv = dinv.as<double2>();
    a.swaps = swaps.as<int32_t>();
    a.rowat = inverse ? rowat.as<int32_t>() : nullptr;
    a.info = info_dev;
    int G = (n - k + kGroup - 1) / kGroup, cur = 0;
    a.cand_in = nullptr;
    a.cand_len = 0;
    a.nsel_groups = G;
    a.final_round = G == 1;
    a.cand_out = cand[cur]->as<int32_t>();
    hipLaunchKernelGGL(gj_select_kernel, dim3((unsigned)(G + (k + kGroup - 1) / kGroup), (unsigned)nmat),
                       dim3(kGroup), 0, s, a);
    CBFM_HIP(hipGetLastError());
    while (G > 1) {
      const int len = G * kW, G2 = (len + kGroup - 1) / kGroup;
      a.cand_in = cand[cur]->as<int32_t>();
      a.cand_len = len;
      a.nsel_groups = G2;
      a.final_round = G2 == 1;
      a.cand_out = cand[1 - cur]->as<int32_t>();
      hipLaunchKernelGGL(gj_select_kernel, dim3((unsigned)G2, (unsigned)nmat), dim3(kGroup), 0, s, a);
      CBFM_HIP(hipGetLastError());
      cur = 1 - cur;
      G = G2;
    }
    RowsArgs r{};
    r.A = A;
    r.strideA = strideA;
    r.ld = ld;
    r.ncols = ncols;
    r.k = k;
    r.w = w;
    r.col0 = inverse ? 0 : k + w;
    r.Dinv = dinv.as<double2>();
    r.swaps = swaps.as<int32_t>();
    const int nchunks = (ncols - r.col0 + kChunk - 1) / kChunk;
    if (nchunks > 0) {
      hipLaunchKernelGGL(gj_rows_kernel, dim3((unsigned)nchunks, (unsigned)nmat), dim3(256), 0, s, r);
      CBFM_HIP(hipGetLastError());
    }
    plan.launch((size_t)st, s);
  }
  if (!inverse) return;
  // column j of the inverse sits at the position that holds input row j
  const int64_t total = (int64_t)nmat * n;
  Scratch src((size_t)total * sizeof(int32_t), s), tmp((size_t)nmat * strideA * sizeof(double2), s);
  CBFM_HIP(hipMemsetAsync(src.p, 0, (size_t)total * sizeof(int32_t), s));
  hipLaunchKernelGGL(gj_src_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rowat.as<int32_t>(),
                     src.as<int32_t>(), n, total);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)nmat), dim3(256), 0,
                     s, A, tmp.as<double2>(), src.as<int32_t>(), n, strideA);
  CBFM_HIP(hipGetLastError());
  CBFM_HIP(hipMemcpyAsync(A, tmp.p, (size_t)nmat * strideA * sizeof(double2), hipMemcpyDeviceToDevice, s));
}

}  // namespace

void gj_check(const int32_t* info_dev, int nmat, const char* what, hipStream_t s) {
  std::vector<int32_t> info(nmat);
  CBFM_HIP(hipMemcpyAsync(info.data(), info_dev, (size_t)nmat * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CBFM_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < nmat; ++b)
    CBFM_REQUIRE(info[b] == 0, CBFM_E_RANK,
                 std::string(what) + (nmat > 1 ? " " + std::to_string(b) : std::string()) +
                     " is singular (no nonzero pivot in column " + std::to_string(info[b] - 1) + ")");
}

void gj_inverse_batched_async(double2* A, int64_t strideA, int n, int nmat, int32_t* info_dev, hipStream_t s) {
  CBFM_REQUIRE(strideA == (int64_t)n * n, CBFM_E_ARG, "Gauss-Jordan inversion: matrices must be packed");
  eliminate(A, strideA, n, n, n, nmat, true, info_dev, s);
}

void gj_inverse_batched(double2* A, int64_t strideA, int n, int nmat, const char* what, hipStream_t s) {
  Scratch info((size_t)std::max(1, nmat) * sizeof(int32_t), s);
  gj_inverse_batched_async(A, strideA, n, nmat, info.as<int32_t>(), s);
  gj_check(info.as<int32_t>(), nmat, what, s);
}

void gj_solve_batched(double2* A, int64_t strideA, int64_t ld, int n, int ncols, int nmat, const char* what,
                      hipStream_t s) {
  CBFM_REQUIRE(ncols > n, CBFM_E_ARG, "Gauss-Jordan solve: no right-hand side");
  Scratch info((size_t)std::max(1, nmat) * sizeof(int32_t), s);
  eliminate(A, strideA, ld, n, ncols, nmat, false, info.as<int32_t>(), s);
  gj_check(info.as<int32_t>(), nmat, what, s);
}

}  // namespace cbfm
