// Batched, variable-size complex double GEMM on the gfx950 matrix cores:
//   C = alpha * op(A) * op(B) (+ C if accumulate)
// op in {N, T (transpose), C (conjugate transpose), R (conjugate)}, all
// matrices row-major complex double with leading dimensions.
//
// A wavefront computes a 16 x 16 tile of C with v_mfma_f64_16x16x4_f64
// (real): for each group of 16 k it does 4 x 4 MFMAs, the four real
// products Ar*Br, -Ai*Bi, Ar*Bi, Ai*Br.  In step t = 0..3 lane L holds
// A[L % 16][k] and B[k][L % 16] for k = k0 + 4 t + L / 16 (any assignment
// of the 16 k values to (slot, step) works as long as A and B agree); the
// operands reach that layout through LDS (see zgemm_batched_kernel).
// The accumulator element r of lane L is C[4 r + L / 16][L % 16] (measured
// on gfx950 with indexed operands: rows are interleaved across the four
// lane groups).
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"
#include "gemm.h"

namespace cbfm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Loads through a global-address-space pointer: the compiler then emits
// global instead of flat loads.  Flat loads also count as LDS operations, so
// with them in flight every LDS wait of the K loop would wait for memory.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_global(const double2* p) {
  const d2v w = *(const __attribute__((address_space(1))) d2v*)p;
  return make_double2(w.x, w.y);
}
__device__ __forceinline__ float2 ld_global(const float2* p) {
  const f2v w = *(const __attribute__((address_space(1))) f2v*)p;
  return make_float2(w.x, w.y);
}

// Loads outside an operand read this zero instead (the address is chosen,
// never the value: a value chosen after an unconditional load lets the
// compiler move the load under a branch, one wait per load).
__device__ double2 g_zero2[1];

// 8 bytes (a complex float) loaded from global memory into a double's bits
__device__ __forceinline__ double ld_global8(const void* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}
__device__ __forceinline__ float2 bits_to_float2(double x) {
  union {
    double d;
    float f[2];
  } u;
  u.d = x;
  return make_float2(u.f[0], u.f[1]);
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(x & 0xffffffff));
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Work unit of block b when one product's units (row of tiles, K part) x
// column tile are numbered column fastest: blocks go to the 8 XCDs in
// turn, so within each run of 8 ntn blocks the ntn column tiles of a row
// and K part go to blocks 8 apart, which one XCD runs one after the other,
// sharing that part of op(A)'s rows in its L2 (read from HBM once instead
// of ntn times).  A bijection of [0, units); the last partial run is kept.
__device__ __forceinline__ int64_t xcd_unit(int64_t b, int64_t units, int64_t ntn) {
  const int64_t run = 8 * ntn, full = units / run * run;
  if (b >= full) return b;
  const int64_t base = b / run * run, r = b - base;
  return base + (r % 8) * ntn + r / 8;
}

// C (tile at rows m0.., columns n0..; CT column blocks) = alpha (cr + i ci),
// or added to C, in the accumulator layout of the FP64 matrix cores.
template <int CT>
__device__ __forceinline__ void store_tile(const GemmDesc& d, int64_t m0, int64_t n0, int lane, const dbl4 (&cr)[CT],
                                           const dbl4 (&ci)[CT]) {
  const int slot = lane >> 4;
#pragma unroll
  for (int u = 0; u < CT; ++u) {
    const int64_t col = n0 + 16 * u + (lane & 15);
    if (col >= d.N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + 4 * r + slot;
      if (row < d.M) {
        const double xr = cr[u][r], xi = ci[u][r];
        double2 v = make_double2(d.alpha_re * xr - d.alpha_im * xi, d.alpha_re * xi + d.alpha_im * xr);
        double2* p = d.transC ? d.C + col * d.ldc + row : d.C + row * d.ldc + col;
        if (d.accumulate) {
          const double2 o = ld_global(p);
          v.x += o.x;
          v.y += o.y;
        }
        *p = v;
      }
    }
  }
}

// SPLITK = 1: each of the 4 wavefronts of a block owns a tile.
// SPLITK > 1: the SPLITK wavefronts of a block share one tile, each taking
// every SPLITK-th group of 16 k, and the partial tiles are summed through
// LDS (few, deep tiles: more loads in flight per tile).
// KB > 1 (SPLITK > 1, one descriptor only): KB consecutive blocks share a
// tile, block b of them taking the groups g with g / SPLITK = b mod KB, so
// that a product of few tiles and long K still has short K loops and fills
// the chip; each block leaves its partial tile in ws (KB x 64 lanes x 8 CT
// doubles per tile) and splitk_reduce_kernel adds them in block order.
// CT > 1 (one descriptor only): a tile is 16 rows by CT adjacent 16-column
// blocks, so a wavefront loads each part of op(A) once for CT column blocks
// (a matrix times a few vectors reads the matrix once instead of CT times).
// Operands go through LDS: each wavefront loads its 16 x 16 sub-tiles of
// op(A) and op(B) along the operand's contiguous dimension (16 lanes x 16 B
// = 256 B per row or column of memory), writes them to its own LDS region
// and reads them back in the matrix-core layout.  Loading the matrix-core
// layout straight from memory spreads every load instruction over 32 cache
// lines and runs at about half the speed on the shapes of this library.
// (Tiles of one column block keep to 128 registers, 4 wavefronts per SIMD,
// so that a few-tile product's blocks all fit on the chip at once.)
template <int SPLITK, int CT>
__global__ void __launch_bounds__(SPLITK == 1 ? 256 : 64 * SPLITK, CT == 1 ? 4 : 1)
    zgemm_batched_kernel(const GemmDesc* __restrict__ desc, int ndesc, int64_t total_tiles, int KB = 1,
                         double* __restrict__ ws = nullptr) {
  constexpr int NW = SPLITK == 1 ? 4 : SPLITK;  // wavefronts per block
  constexpr int NS = 1 + CT;                    // staged sub-tiles per wavefront: A, then B per column block
  constexpr int STAGE = NW * NS * 16 * 17;      // double2, rows padded to 17
  constexpr int RED = SPLITK == 1 ? 0 : (SPLITK - 1) * 64 * 4 * CT;  // double2: partial tiles of waves 1..
  // the split-K partial sums reuse the staging memory after the K loop
  __shared__ double2 smem[STAGE > RED ? STAGE : RED];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // wave-uniform tile and descriptor (readfirstlane makes the K loop a scalar
  // loop: the accumulators then stay in the matrix-core registers across it)
  int64_t tile = SPLITK == 1 ? (int64_t)blockIdx.x * 4 + wave : (int64_t)blockIdx.x / KB;
  int kb = SPLITK == 1 ? 0 : (int)(blockIdx.x % KB);
  if (SPLITK > 1 && ndesc == 1) {  // one product, a tile (or K part) per block: XCD-aware order
    const int64_t ntn0 = (uniform64(desc[0].N) + 16 * CT - 1) / (16 * CT);
    const int64_t u = xcd_unit(blockIdx.x, total_tiles * KB, ntn0), rk = u / ntn0;
    tile = (rk / KB) * ntn0 + u % ntn0;
    kb = (int)(rk % KB);
  }
  if (tile >= total_tiles) return;  // uniform per block when SPLITK > 1
  // descriptor holding this tile (tile_start ascending)
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile_start <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  GemmDesc d = desc[lo];
  // the descriptor is wave-uniform: keep its sizes in scalar registers
  d.M = uniform64(d.M);
  d.N = uniform64(d.N);
  d.K = uniform64(d.K);
  d.lda = uniform64(d.lda);
  d.ldb = uniform64(d.ldb);
  d.ldc = uniform64(d.ldc);
  d.tile_start = uniform64(d.tile_start);
  d.opA = __builtin_amdgcn_readfirstlane(d.opA);
  d.opB = __builtin_amdgcn_readfirstlane(d.opB);
  const int64_t t = tile - (CT == 1 ? d.tile_start : 0);
  const int64_t ntn = (d.N + 16 * CT - 1) / (16 * CT);
  const int64_t m0 = (t / ntn) * 16, n0 = (t % ntn) * 16 * CT;
  const int slot = lane >> 4, li = lane & 15;
  // which operand dimension is contiguous in memory
  const bool a_k = d.opA == OP_N || d.opA == OP_R;  // A[i][k] at i lda + k
  const bool b_k = d.opB == OP_T || d.opB == OP_C;  // B[k][j] at j ldb + k
  // complex products with three real products (3M): over this wave's k,
  // p1 = sum ar br, p2 = sum ai bi, p3 = sum (ar + ai)(br + bi); then
  // re = p1 - p2 and im = p3 - p1 - p2 (normwise as accurate as the
  // four-product form, with a quarter fewer matrix-core operations)
  dbl4 p1[CT], p2[CT], p3[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) p1[u] = p2[u] = p3[u] = dbl4{0, 0, 0, 0};
  // this wavefront's groups of 16 k: k0 = 16 (wave + SPLITK g), g < ng
  const int64_t kfirst = SPLITK == 1 ? 0 : 16 * (wave + (int64_t)SPLITK * kb), kstep = 16 * SPLITK * KB;
  const int64_t ng = kfirst < d.K ? (d.K - kfirst + kstep - 1) / kstep : 0;
  double2 ga[4], gb[CT][4];
  // Lane (slot, li), load q: line 4 q + slot of the operand, element li
  // along it, i.e. op(A)[m0 + ar][k + ak] and op(B)[k + bk][n0 + 16 u + bc]
  // for the group starting at k.  Each load walks its line of memory with a
  // fixed element step per group; off* is its element offset and n* the
  // number of groups it stays inside the matrix (loads past it read zero).
  const int64_t sAk = a_k ? 1 : d.lda, sAi = a_k ? d.lda : 1;
  const int64_t sBk = b_k ? 1 : d.ldb, sBj = b_k ? d.ldb : 1;
  const double sgA = (d.opA == OP_C || d.opA == OP_R) ? -1.0 : 1.0;
  const double sgB = (d.opB == OP_C || d.opB == OP_R) ? -1.0 : 1.0;
  const int64_t stA = kstep * sAk, stB = kstep * sBk;
  int ar[4], ak[4], bk[4], bc[4];
  int64_t offA[4], nA[4], offB[CT][4], nB[CT][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + slot;
    ar[q] = a_k ? r : li;
    ak[q] = a_k ? li : r;
    bk[q] = b_k ? li : r;
    bc[q] = b_k ? r : li;
    const int64_t i = m0 + ar[q], ka = kfirst + ak[q], kb = kfirst + bk[q];
    nA[q] = i < d.M && ka < d.K ? (d.K - ka + kstep - 1) / kstep : 0;
    offA[q] = nA[q] > 0 ? i * sAi + ka * sAk : 0;
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const int64_t j = n0 + 16 * u + bc[q];
      nB[u][q] = j < d.N && kb < d.K ? (d.K - kb + kstep - 1) / kstep : 0;
      offB[u][q] = nB[u][q] > 0 ? j * sBj + kb * sBk : 0;
    }
  }
  auto gload = [&](int64_t g) {  // group g; called for g = 0, 1, 2, ... in order
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ga[q] = ld_global(g < nA[q] ? d.A + offA[q] : g_zero2);
      offA[q] += stA;
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        gb[u][q] = ld_global(g < nB[u][q] ? d.B + offB[u][q] : g_zero2);
        offB[u][q] += stB;
      }
    }
  };
  // this wavefront's staging: sub-tile 0 = op(A) rows x k, 1 + u = op(B) columns of block u x k
  double2(*st)[16][17] = reinterpret_cast<double2(*)[16][17]>(smem + (size_t)wave * NS * 16 * 17);
  if (ng > 0) gload(0);
  for (int64_t g = 0; g < ng; ++g) {
    // (the conjugation sign is applied here, where the loads are waited on)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      st[0][ar[q]][ak[q]] = make_double2(ga[q].x, sgA * ga[q].y);
#pragma unroll
      for (int u = 0; u < CT; ++u) st[1 + u][bc[q]][bk[q]] = make_double2(gb[u][q].x, sgB * gb[u][q].y);
    }
    // the next group's loads go out before the matrix cores take this one
    // (unconditionally: past the last group they read zeros, and a
    // conditional load would leave register copies that wait on it)
    gload(g + 1);
    // LDS operations of a wavefront complete in order: a compiler barrier
    // keeps the reads after the writes (and the next writes after the reads)
    __builtin_amdgcn_wave_barrier();
    double2 a[4], b[CT][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {  // step s takes k = 4 s + slot
      a[s] = st[0][li][4 * s + slot];
#pragma unroll
      for (int u = 0; u < CT; ++u) b[u][s] = st[1 + u][li][4 * s + slot];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < CT; ++u) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        p1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].x, b[u][s].x, p1[u], 0, 0, 0);
        p2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].y, b[u][s].y, p2[u], 0, 0, 0);
        p3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].x + a[s].y, b[u][s].x + b[u][s].y, p3[u], 0, 0, 0);
      }
    }
  }
  dbl4 cr[CT], ci[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cr[u][q] = p1[u][q] - p2[u][q];
      ci[u][q] = p3[u][q] - p1[u][q] - p2[u][q];
    }
  if (SPLITK > 1) {
    // waves 1..SPLITK-1 hand their partial tiles to wave 0 (through the
    // staging memory: every wavefront has left the K loop first)
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    if (wave > 0) {
      double* r = red + ((wave - 1) * 64 + lane) * 8 * CT;
#pragma unroll
      for (int u = 0; u < CT; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          r[8 * u + q] = cr[u][q];
          r[8 * u + 4 + q] = ci[u][q];
        }
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < SPLITK - 1; ++w) {
      const double* r = red + (w * 64 + lane) * 8 * CT;
#pragma unroll
      for (int u = 0; u < CT; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          cr[u][q] += r[8 * u + q];
          ci[u][q] += r[8 * u + 4 + q];
        }
    }
    if (KB > 1) {  // this block's part of the tile, for splitk_reduce_kernel
      double* o = ws + (((int64_t)tile * KB + kb) * 64 + lane) * 8 * CT;
#pragma unroll
      for (int u = 0; u < CT; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          o[8 * u + q] = cr[u][q];
          o[8 * u + 4 + q] = ci[u][q];
        }
      return;
    }
  }
  store_tile<CT>(d, m0, n0, lane, cr, ci);
}

// The tiles of a K-split product (one descriptor): a block of four
// wavefronts per tile, wavefront w adding the parts b = w, w + 4, ... from
// ws (its loads all in flight), then wavefront 0 adding the four sums in
// order through LDS and storing the tile.  With at most four parts this is
// the block order.
template <int CT>
__global__ void __launch_bounds__(256)
    splitk_reduce_kernel(const GemmDesc* __restrict__ desc, int64_t total_tiles, int KB, const double* __restrict__ ws) {
  const int64_t tile = blockIdx.x;
  if (tile >= total_tiles) return;  // uniform per block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const GemmDesc d = desc[0];
  const int64_t t = tile - (CT == 1 ? d.tile_start : 0);
  const int64_t ntn = (d.N + 16 * CT - 1) / (16 * CT);
  const int64_t m0 = (t / ntn) * 16, n0 = (t % ntn) * 16 * CT;
  dbl4 cr[CT], ci[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) cr[u] = ci[u] = dbl4{0, 0, 0, 0};
#pragma unroll 4
  for (int b = wave; b < KB; b += 4) {
    const double* r = ws + ((tile * KB + b) * 64 + lane) * 8 * CT;
#pragma unroll
    for (int u = 0; u < CT; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cr[u][q] += r[8 * u + q];
        ci[u][q] += r[8 * u + 4 + q];
      }
  }
  __shared__ double part[3][8 * CT][64];
  if (wave > 0) {
#pragma unroll
    for (int u = 0; u < CT; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        part[wave - 1][8 * u + q][lane] = cr[u][q];
        part[wave - 1][8 * u + 4 + q][lane] = ci[u][q];
      }
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int u = 0; u < CT; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cr[u][q] += part[w][8 * u + q][lane];
        ci[u][q] += part[w][8 * u + 4 + q][lane];
      }
  store_tile<CT>(d, m0, n0, lane, cr, ci);
}

// ------------------------------------------------------------------------
// FP32 / BF16 matrix cores (FP32 accumulation).  v_mfma_f32_16x16x4f32 and
// v_mfma_f32_16x16x32_bf16 take A[L % 16][k] and B[k][L % 16] in lane L for
// the k of the lane's slot L / 16 (one k per slot in FP32, eight
// consecutive k per slot in BF16); their accumulator element r of lane L is
// C[4 (L / 16) + r][L % 16] (measured on gfx950; unlike the FP64
// instruction, the four rows of a lane are consecutive).
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int MODE, int SPLITK, bool A64, bool B64>
__global__ void __launch_bounds__(256) xgemm_batched_kernel(const GemmDescX* __restrict__ desc, int ndesc,
                                                            int64_t total_tiles) {
  constexpr int KG = MODE == XG_FP32 ? 16 : 32;  // k per step of a wavefront
  constexpr int NW = SPLITK == 1 ? 4 : SPLITK;   // wavefronts per block
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tile = SPLITK == 1 ? (int64_t)blockIdx.x * 4 + wave : (int64_t)blockIdx.x;
  // operands staged through LDS as in zgemm_batched_kernel, as complex float
  __shared__ float2 stage[NW][2][16][KG + 1];
  __shared__ float red[SPLITK == 1 ? 1 : (SPLITK - 1) * 64 * 8];
  if (tile >= total_tiles) return;  // uniform per block when SPLITK > 1
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile_start <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  GemmDescX d = desc[lo];
  d.M = uniform64(d.M);
  d.N = uniform64(d.N);
  d.K = uniform64(d.K);
  d.lda = uniform64(d.lda);
  d.ldb = uniform64(d.ldb);
  d.ldc = uniform64(d.ldc);
  d.tile_start = uniform64(d.tile_start);
  d.opA = __builtin_amdgcn_readfirstlane(d.opA);
  d.opB = __builtin_amdgcn_readfirstlane(d.opB);
  const int64_t t = tile - d.tile_start;
  const int64_t ntn = (d.N + 15) / 16;
  const int64_t m0 = (t / ntn) * 16, n0 = (t % ntn) * 16;
  const int slot = lane >> 4, li = lane & 15;
  const bool a_k = d.opA == OP_N || d.opA == OP_R;  // A[i][k] at i lda + k
  const bool b_k = d.opB == OP_T || d.opB == OP_C;  // B[k][j] at j ldb + k
  // lane (slot, li), load q: line 4 q + slot of the operand, element li
  // along it, walked with a fixed element step per step of k as in
  // zgemm_batched_kernel; operands of complex double are rounded to float
  const int64_t kfirst = SPLITK == 1 ? 0 : (int64_t)KG * wave, kstep = (int64_t)KG * SPLITK;
  const int64_t sAk = a_k ? 1 : d.lda, sAi = a_k ? d.lda : 1;
  const int64_t sBk = b_k ? 1 : d.ldb, sBj = b_k ? d.ldb : 1;
  const float sgA = (d.opA == OP_C || d.opA == OP_R) ? -1.0f : 1.0f;
  const float sgB = (d.opB == OP_C || d.opB == OP_R) ? -1.0f : 1.0f;
  int ar[4], ak[4], bk[4], bc[4];
  int64_t offA[4], offB[4], kA[4], kB[4];
  bool rA[4], rB[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + slot;
    ar[q] = a_k ? r : li;
    ak[q] = a_k ? li : r;
    bk[q] = b_k ? li : r;
    bc[q] = b_k ? r : li;
    const int64_t i = m0 + ar[q], j = n0 + bc[q];
    rA[q] = i < d.M;
    rB[q] = j < d.N;
    kA[q] = kfirst + ak[q];
    kB[q] = kfirst + bk[q];
    offA[q] = rA[q] ? i * sAi + kA[q] * sAk : 0;
    offB[q] = rB[q] ? j * sBj + kB[q] * sBk : 0;
  }
  float2(*sa)[KG + 1] = stage[wave][0];
  float2(*sb)[KG + 1] = stage[wave][1];
  flt4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  // raw operand values of one step (half h, load q): a complex double, or
  // the 8 bytes of a complex float in .x.  The next step's loads go out
  // before this one's matrix-core work; loads outside an operand read zero
  // (the address is chosen, not the value, as in zgemm_batched_kernel), and
  // the conversion and the conjugation sign are applied at the LDS store.
  double2 ra[KG / 16][4], rb[KG / 16][4];
  auto gload = [&]() {  // the step at the running offsets, which it advances
    if constexpr (A64) {
#pragma unroll
      for (int h = 0; h < KG / 16; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          ra[h][q] = ld_global(rA[q] && kA[q] + 16 * h < d.K
                                   ? static_cast<const double2*>(d.A) + offA[q] + 16 * h * sAk
                                   : g_zero2);
    } else {
#pragma unroll
      for (int h = 0; h < KG / 16; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          ra[h][q].x = ld_global8(rA[q] && kA[q] + 16 * h < d.K
                                      ? (const void*)(static_cast<const float2*>(d.A) + offA[q] + 16 * h * sAk)
                                      : (const void*)g_zero2);
    }
    if constexpr (B64) {
#pragma unroll
      for (int h = 0; h < KG / 16; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          rb[h][q] = ld_global(rB[q] && kB[q] + 16 * h < d.K
                                   ? static_cast<const double2*>(d.B) + offB[q] + 16 * h * sBk
                                   : g_zero2);
    } else {
#pragma unroll
      for (int h = 0; h < KG / 16; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          rb[h][q].x = ld_global8(rB[q] && kB[q] + 16 * h < d.K
                                      ? (const void*)(static_cast<const float2*>(d.B) + offB[q] + 16 * h * sBk)
                                      : (const void*)g_zero2);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      kA[q] += kstep;
      kB[q] += kstep;
      offA[q] += kstep * sAk;
      offB[q] += kstep * sBk;
    }
  };
  if (kfirst < d.K) gload();
  for (int64_t k0 = kfirst; k0 < d.K; k0 += kstep) {
#pragma unroll
    for (int h = 0; h < KG / 16; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float2 va = A64 ? make_float2((float)ra[h][q].x, (float)ra[h][q].y) : bits_to_float2(ra[h][q].x);
        const float2 vb = B64 ? make_float2((float)rb[h][q].x, (float)rb[h][q].y) : bits_to_float2(rb[h][q].x);
        sa[ar[q]][16 * h + ak[q]] = make_float2(va.x, sgA * va.y);
        sb[bc[q]][16 * h + bk[q]] = make_float2(vb.x, sgB * vb.y);
      }
    gload();  // the next step (zeros past the end)
    // LDS operations of a wavefront complete in order
    __builtin_amdgcn_wave_barrier();
    if constexpr (MODE == XG_FP32) {
      float2 a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // step q takes k = 4 q + slot
        a[q] = sa[li][4 * q + slot];
        b[q] = sb[li][4 * q + slot];
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].x, b[q].x, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[q].y, b[q].y, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].x, b[q].y, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].y, b[q].x, ci, 0, 0, 0);
      }
    } else if constexpr (MODE == XG_BF16) {
      bf16x8 ar, ai, an, br, bi;
#pragma unroll
      for (int q = 0; q < 8; ++q) {  // slot takes k = 8 slot + q
        const float2 a = sa[li][8 * slot + q];
        const float2 b = sb[li][8 * slot + q];
        ar[q] = (__bf16)a.x;
        ai[q] = (__bf16)a.y;
        an[q] = (__bf16)(-a.y);
        br[q] = (__bf16)b.x;
        bi[q] = (__bf16)b.y;
      }
      __builtin_amdgcn_wave_barrier();
      cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(an, bi, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, ci, 0, 0, 0);
    } else {
      // split BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); the
      // products hi*hi + hi*lo + lo*hi keep about 16 significant bits
      bf16x8 arh, arl, aih, ail, anh, anl, brh, brl, bih, bil;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float2 a = sa[li][8 * slot + q];
        const float2 b = sb[li][8 * slot + q];
        arh[q] = (__bf16)a.x;
        arl[q] = (__bf16)(a.x - (float)arh[q]);
        aih[q] = (__bf16)a.y;
        ail[q] = (__bf16)(a.y - (float)aih[q]);
        anh[q] = -aih[q];
        anl[q] = -ail[q];
        brh[q] = (__bf16)b.x;
        brl[q] = (__bf16)(b.x - (float)brh[q]);
        bih[q] = (__bf16)b.y;
        bil[q] = (__bf16)(b.y - (float)bih[q]);
      }
      __builtin_amdgcn_wave_barrier();
#define XG_SPLIT3(acc, xh, xl, yh, yl)                                  \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0); \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0); \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);
      XG_SPLIT3(cr, arh, arl, brh, brl)
      XG_SPLIT3(cr, anh, anl, bih, bil)
      XG_SPLIT3(ci, arh, arl, bih, bil)
      XG_SPLIT3(ci, aih, ail, brh, brl)
#undef XG_SPLIT3
    }
  }
  if (SPLITK > 1) {
    if (wave > 0) {
      float* r = red + ((wave - 1) * 64 + lane) * 8;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        r[q] = cr[q];
        r[4 + q] = ci[q];
      }
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < SPLITK - 1; ++w) {
      const float* r = red + (w * 64 + lane) * 8;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cr[q] += r[q];
        ci[q] += r[4 + q];
      }
    }
  }
  const int64_t col = n0 + (lane & 15);
  if (col >= d.N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = m0 + 4 * slot + r;
    if (row < d.M) {
      const float xr = cr[r], xi = ci[r];
      const float vr = d.alpha_re * xr - d.alpha_im * xi, vi = d.alpha_re * xi + d.alpha_im * xr;
      const int64_t off = d.transC ? col * d.ldc + row : row * d.ldc + col;
      if (d.c64)
        static_cast<double2*>(d.C)[off] = make_double2(vr, vi);
      else
        static_cast<float2*>(d.C)[off] = make_float2(vr, vi);
    }
  }
}

static int64_t number_tiles_x(const std::vector<GemmDescX>& in, std::vector<GemmDescX>& out, double* flops) {
  int64_t tiles = 0;
  for (GemmDescX d : in) {
    CBFM_REQUIRE(d.M >= 0 && d.N >= 0 && d.K >= 0, CBFM_E_ARG, "negative GEMM size");
    if (d.M == 0 || d.N == 0) continue;
    d.tile_start = tiles;
    tiles += ((d.M + 15) / 16) * ((d.N + 15) / 16);
    *flops += 8.0 * (double)d.M * (double)d.N * (double)d.K;
    out.push_back(d);
  }
  return tiles;
}

// Element types of a group's operands (bit 1: A is complex double, bit 0:
// B is); every product of one launch has the same pair, which the kernel
// takes as template arguments so that its loads carry no run-time choice.
static int operand_types(const GemmDescX* g, size_t count) {
  if (count == 0) return 0;
  const int ab = (g[0].a64 ? 2 : 0) | (g[0].b64 ? 1 : 0);
  for (size_t i = 0; i < count; ++i)
    CBFM_REQUIRE(((g[i].a64 ? 2 : 0) | (g[i].b64 ? 1 : 0)) == ab, CBFM_E_ARG,
                 "mixed operand element types in one batched GEMM launch");
  return ab;
}

template <int MODE, int SPLITK>
static void launch_x_types(const GemmDescX* dd, int n, int64_t tiles, int ab, dim3 g, hipStream_t s) {
  switch (ab) {
    case 0:
      hipLaunchKernelGGL((xgemm_batched_kernel<MODE, SPLITK, false, false>), g, dim3(256), 0, s, dd, n, tiles);
      break;
    case 1:
      hipLaunchKernelGGL((xgemm_batched_kernel<MODE, SPLITK, false, true>), g, dim3(256), 0, s, dd, n, tiles);
      break;
    case 2:
      hipLaunchKernelGGL((xgemm_batched_kernel<MODE, SPLITK, true, false>), g, dim3(256), 0, s, dd, n, tiles);
      break;
    default:
      hipLaunchKernelGGL((xgemm_batched_kernel<MODE, SPLITK, true, true>), g, dim3(256), 0, s, dd, n, tiles);
  }
}

template <int MODE>
static void launch_x_mode(const GemmDescX* dd, int n, int64_t tiles, int ab, hipStream_t s) {
  const bool few = tiles < 4096;
  const dim3 g(few ? (unsigned)tiles : (unsigned)((tiles + 3) / 4));
  if (few)
    launch_x_types<MODE, 4>(dd, n, tiles, ab, g, s);
  else
    launch_x_types<MODE, 1>(dd, n, tiles, ab, g, s);
}

static void launch_x(const GemmDescX* dd, int n, int64_t tiles, double flops, int mode, int ab, hipStream_t s) {
  TimedLaunch tl(T_XGEMM, s, flops);
  if (mode == XG_BF16)
    launch_x_mode<XG_BF16>(dd, n, tiles, ab, s);
  else if (mode == XG_BF16X3)
    launch_x_mode<XG_BF16X3>(dd, n, tiles, ab, s);
  else
    launch_x_mode<XG_FP32>(dd, n, tiles, ab, s);
  CBFM_HIP(hipGetLastError());
}

void xgemm_batched(std::vector<GemmDescX>& descs, int mode, hipStream_t s,
                   std::vector<std::vector<GemmDescX>>* keep) {
  if (descs.empty()) return;
  std::vector<GemmDescX> live;
  double flops = 0;
  const int64_t tiles = number_tiles_x(descs, live, &flops);
  if (live.empty()) return;
  const int ab = operand_types(live.data(), live.size());
  Scratch dev(live.size() * sizeof(GemmDescX), s);
  CBFM_HIP(hipMemcpyAsync(dev.p, live.data(), live.size() * sizeof(GemmDescX), hipMemcpyHostToDevice, s));
  launch_x(dev.as<GemmDescX>(), (int)live.size(), tiles, flops, mode, ab, s);
  if (keep) {  // the caller keeps the staged descriptors until it synchronises s
    keep->push_back(std::move(live));
    return;
  }
  CBFM_HIP(hipStreamSynchronize(s));  // the descriptor staging buffer is host memory of this frame
}

XGemmPlan::XGemmPlan(const std::vector<std::vector<GemmDescX>>& groups, int mode, hipStream_t s)
    : mode_(mode), dev_(std::max<size_t>(1, [&] {
                          size_t k = 0;
                          for (const auto& g : groups) k += g.size();
                          return k;
                        }()) * sizeof(GemmDescX),
                        s) {
  std::vector<GemmDescX> all;
  for (const auto& g : groups) {
    first_.push_back((int64_t)all.size());
    double f = 0;
    tiles_.push_back(number_tiles_x(g, all, &f));
    flops_.push_back(f);
    count_.push_back((int64_t)all.size() - first_.back());
    types_.push_back(operand_types(all.data() + first_.back(), (size_t)count_.back()));
  }
  if (!all.empty()) {
    CBFM_HIP(hipMemcpyAsync(dev_.p, all.data(), all.size() * sizeof(GemmDescX), hipMemcpyHostToDevice, s));
    CBFM_HIP(hipStreamSynchronize(s));  // `all` is host memory of this frame
  }
}

void XGemmPlan::launch(size_t g, hipStream_t s) const {
  CBFM_REQUIRE(g < tiles_.size(), CBFM_E_ARG, "GEMM plan group out of range");
  if (count_[g] == 0) return;
  launch_x(dev_.as<GemmDescX>() + first_[g], (int)count_[g], tiles_[g], flops_[g], mode_, types_[g], s);
}

// Tile offsets of a group of descriptors (empty products dropped); returns
// the group's tile count.
static int64_t number_tiles(const std::vector<GemmDesc>& in, std::vector<GemmDesc>& out, double* flops) {
  int64_t tiles = 0;
  for (GemmDesc d : in) {
    CBFM_REQUIRE(d.M >= 0 && d.N >= 0 && d.K >= 0, CBFM_E_ARG, "negative GEMM size");
    if (d.M == 0 || d.N == 0) continue;
    d.tile_start = tiles;
    tiles += ((d.M + 15) / 16) * ((d.N + 15) / 16);
    *flops += 8.0 * (double)d.M * (double)d.N * (double)d.K;  // complex multiply-add = 8 real flops
    out.push_back(d);
  }
  return tiles;
}

// A single matrix-vector product (N = 1, rows of op(A) contiguous: op N or
// conj) on the vector units: the tiled kernels would pad the one column to
// 16 and spend sixteen times the matrix-core work.  One wavefront per row,
// lanes along the row, four loads in flight per lane, the row sum by a
// butterfly; alpha and accumulation as in the tiled kernel.
__global__ void __launch_bounds__(256) zgemv_kernel(const GemmDesc* __restrict__ desc) {
  const int lane = threadIdx.x & 63;
  GemmDesc d = desc[0];
  d.M = uniform64(d.M);
  d.K = uniform64(d.K);
  d.lda = uniform64(d.lda);
  d.ldb = uniform64(d.ldb);
  d.ldc = uniform64(d.ldc);
  d.opA = __builtin_amdgcn_readfirstlane(d.opA);
  d.opB = __builtin_amdgcn_readfirstlane(d.opB);
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= d.M) return;  // uniform over the wavefront
  const double sgA = d.opA == OP_R ? -1.0 : 1.0;
  const double sgB = (d.opB == OP_C || d.opB == OP_R) ? -1.0 : 1.0;
  const int64_t sx = (d.opB == OP_T || d.opB == OP_C) ? 1 : d.ldb;  // x_k = B[k sx]
  const double2* ar = d.A + row * d.lda;
  double re = 0, im = 0;
  for (int64_t k0 = lane; k0 < d.K; k0 += 256) {
    double2 a[4], x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + 64 * u;
      a[u] = ld_global(k < d.K ? ar + k : g_zero2);
      x[u] = ld_global(k < d.K ? d.B + k * sx : g_zero2);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double ax = a[u].x, ay = sgA * a[u].y, xx = x[u].x, xy = sgB * x[u].y;
      re += ax * xx - ay * xy;
      im += ax * xy + ay * xx;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    double2 v = make_double2(d.alpha_re * re - d.alpha_im * im, d.alpha_re * im + d.alpha_im * re);
    double2* p = d.transC ? d.C + row : d.C + row * d.ldc;  // column 0
    if (d.accumulate) {
      const double2 o = ld_global(p);
      v.x += o.x;
      v.y += o.y;
    }
    *p = v;
  }
}

// A product with at most 16 CT columns, op(A) rows and op(B) columns
// contiguous along k (such as the GMRES matrix times a block of vectors),
// or nb such products whose operands and results lie sA, sB, sC elements
// apart (one per right-hand side): a block of four wavefronts takes 64 rows
// of op(A), 16 per wavefront, against all 16 CT columns, over a contiguous
// range of the K groups (block kb of KB for its rows).  op(A) is read once.
// Each group's 16 k x 16 CT columns of op(B) are loaded once per block and
// shared by the four wavefronts through LDS (two buffers, so one barrier
// per group), where the tiled kernels load them once per 16 x 16 tile.
// Every wavefront holds the raw operands of two groups in flight.  The
// partial tiles go to ws in splitk_reduce_kernel<CT>'s layout (the tile of
// wavefront w of row block p of product c is c T + 4 p + w, T tiles per
// product); panel_reduce_kernel adds them in block order and stores C.
template <int CT>
__global__ void __launch_bounds__(256, CT == 1 ? 4 : 3)
    zgemm_panel_kernel(const GemmDesc* __restrict__ desc, int KB, double* __restrict__ ws, int64_t sA, int64_t sB) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slot = lane >> 4, li = lane & 15;
  GemmDesc d = desc[0];
  d.M = uniform64(d.M);
  d.N = uniform64(d.N);
  d.K = uniform64(d.K);
  d.lda = uniform64(d.lda);
  d.ldb = uniform64(d.ldb);
  d.opA = __builtin_amdgcn_readfirstlane(d.opA);
  d.opB = __builtin_amdgcn_readfirstlane(d.opB);
  const int64_t nrb = (d.M + 63) / 64;
  const int64_t c = blockIdx.x / (nrb * KB), rb = blockIdx.x / KB % nrb;
  const int kb = (int)(blockIdx.x % KB);
  d.A += c * sA;
  d.B += c * sB;
  const int64_t G = (d.K + 15) / 16;
  const int64_t g0 = G * kb / KB, g1 = G * (kb + 1) / KB;  // this block's groups of 16 k
  const int64_t m0 = rb * 64 + 16 * wave;
  const double sgA = d.opA == OP_R ? -1.0 : 1.0;
  const double sgB = d.opB == OP_C ? -1.0 : 1.0;
  // op(A): lane (slot, li), load q reads row m0 + 4 q + slot at k = 16 g + li;
  // op(B): thread t, load h reads column 16 h + t / 16 at k = 16 g + t % 16.
  // Rows past M and columns past N read row M - 1 and column N - 1: they
  // only reach results that are not stored.
  const double2* pA[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) pA[q] = d.A + std::min<int64_t>(m0 + 4 * q + slot, d.M - 1) * d.lda + li;
  const int tc = threadIdx.x >> 4, tk = threadIdx.x & 15;
  const double2* pB[CT];
#pragma unroll
  for (int h = 0; h < CT; ++h) pB[h] = d.B + std::min<int64_t>(16 * h + tc, d.N - 1) * d.ldb + tk;
  // whole groups (every k inside K) load without conditions, so that the
  // waits of the loop count the loads of the group in flight exactly; the
  // last group of a K that is not a multiple of 16 is taken after the loop
  const int64_t ge = std::min(g1, d.K / 16);
  auto gload = [&](int64_t g, double2(&ra)[4], double2(&rbv)[CT]) {
    const int64_t k0 = 16 * g;
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = ld_global(pA[q] + k0);
#pragma unroll
    for (int h = 0; h < CT; ++h) rbv[h] = ld_global(pB[h] + k0);
  };
  __shared__ double2 sa[4][16][17];       // per wavefront: op(A) rows x k
  __shared__ double2 sb[2][16 * CT][17];  // per block, two buffers: op(B) columns x k
  double2(*as)[17] = sa[wave];
  auto put = [&](const double2(&ra)[4], const double2(&rbv)[CT], int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) as[4 * q + slot][li] = make_double2(ra[q].x, sgA * ra[q].y);
#pragma unroll
    for (int h = 0; h < CT; ++h) sb[buf][16 * h + tc][tk] = make_double2(rbv[h].x, sgB * rbv[h].y);
  };
  // 3M products as in zgemm_batched_kernel, CT column blocks
  dbl4 p1[CT], p2[CT], p3[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) p1[u] = p2[u] = p3[u] = dbl4{0, 0, 0, 0};
  auto mma = [&](int buf) {
    double2 a[4], b[CT][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {  // step s takes k = 4 s + slot
      a[s] = as[li][4 * s + slot];
#pragma unroll
      for (int u = 0; u < CT; ++u) b[u][s] = sb[buf][16 * u + li][4 * s + slot];
    }
    // the wavefront's next writes of its op(A) rows stay after these reads
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < CT; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        p1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].x, b[u][s].x, p1[u], 0, 0, 0);
        p2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].y, b[u][s].y, p2[u], 0, 0, 0);
        p3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].x + a[s].y, b[u][s].x + b[u][s].y, p3[u], 0, 0, 0);
      }
  };
  // a buffer of sb is rewritten two groups after it was read: every
  // wavefront has passed the barrier of the group in between by then
  int last = 1;  // buffer of the last group taken
  if (g0 < ge) {  // uniform over the block
    double2 ra0[4], rb0[CT], ra1[4], rb1[CT];
    // prefetches past this block's whole groups read its last one again
    gload(g0, ra0, rb0);
    gload(std::min(g0 + 1, ge - 1), ra1, rb1);
    // pairs of groups: the loop is entered and repeated only with both
    // groups' loads in flight, so each wait leaves the other group's loads
    // outstanding
    // (the scheduling barriers keep a group's stores to LDS, which wait on
    // its loads, from being moved above the other group's matrix-core work)
    int64_t g = g0;
    for (; g + 1 < ge; g += 2) {  // g, ge: uniform over the block
      put(ra0, rb0, 0);
      gload(std::min(g + 2, ge - 1), ra0, rb0);
      __syncthreads();
      mma(0);
      __builtin_amdgcn_sched_barrier(0);
      put(ra1, rb1, 1);
      gload(std::min(g + 3, ge - 1), ra1, rb1);
      __syncthreads();
      mma(1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (g < ge) {  // one group left, in ra0
      put(ra0, rb0, 0);
      __syncthreads();
      mma(0);
      last = 0;
    }
  }
  if (d.K % 16 != 0 && g0 <= G - 1 && G - 1 < g1) {  // the partial last group of K, if this block's
    const int64_t k0 = 16 * ge;
    double2 ra[4], rbv[CT];
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = ld_global(k0 + li < d.K ? pA[q] + k0 : g_zero2);
#pragma unroll
    for (int h = 0; h < CT; ++h) rbv[h] = ld_global(k0 + tk < d.K ? pB[h] + k0 : g_zero2);
    put(ra, rbv, 1 - last);
    __syncthreads();
    mma(1 - last);
  }
  const int64_t nt = (d.M + 15) / 16, tile = rb * 4 + wave;
  if (tile >= nt) return;
  double* o = ws + (((c * nt + tile) * KB + kb) * 64 + lane) * 8 * CT;
#pragma unroll
  for (int u = 0; u < CT; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o[8 * u + q] = p1[u][q] - p2[u][q];
      o[8 * u + 4 + q] = p3[u][q] - p1[u][q] - p2[u][q];
    }
}

// The row-block kernel's partial tiles (splitk_reduce_kernel<CT>'s layout;
// nb products, results sC elements apart), one thread per element of C:
// the KB parts added in block order, then alpha and the store as in
// store_tile.  Consecutive threads read one lane's 64 CT bytes of a part.
template <int CT>
__global__ void __launch_bounds__(256) panel_reduce_kernel(const GemmDesc* __restrict__ desc, int64_t total_tiles,
                                                           int KB, const double* __restrict__ ws, int64_t sC) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total_tiles * 256 * CT) return;
  const int64_t gt = e / (256 * CT);  // tile over all products
  const int f = (int)(e % (256 * CT));
  const int lane = f / (4 * CT), u = f / 4 % CT, q = f % 4;
  const GemmDesc d = desc[0];
  const int64_t nt = (d.M + 15) / 16, c = gt / nt;
  const int64_t row = gt % nt * 16 + 4 * q + (lane >> 4), col = 16 * u + (lane & 15);
  const double* r = ws + (gt * KB * 64 + lane) * 8 * CT + 8 * u + q;
  double xr = 0, xi = 0;
#pragma unroll 4
  for (int b = 0; b < KB; ++b) {
    xr += r[(int64_t)b * 64 * 8 * CT];
    xi += r[(int64_t)b * 64 * 8 * CT + 4];
  }
  if (row >= d.M || col >= d.N) return;
  double2 v = make_double2(d.alpha_re * xr - d.alpha_im * xi, d.alpha_re * xi + d.alpha_im * xr);
  double2* p = (d.transC ? d.C + col * d.ldc + row : d.C + row * d.ldc + col) + c * sC;
  if (d.accumulate) {
    const double2 o = ld_global(p);
    v.x += o.x;
    v.y += o.y;
  }
  *p = v;
}

// Blocks per 64 rows of the row-block kernel: `per` blocks over the nb
// products' rows, at most one per group of 16 k.
static int panel_blocks_per_rows(int64_t M, int64_t K, int64_t nb, int64_t per) {
  const int64_t rows = nb * ((M + 63) / 64), groups = std::max<int64_t>(1, (K + 15) / 16);
  return (int)std::max<int64_t>(1, std::min(groups, per / std::max<int64_t>(1, rows)));
}

// Launch shapes: four tiles per block (one per wavefront), or one tile per
// block with K split over 4 or 8 wavefronts; for a single product also
// tiles of 2 or 4 adjacent 16-column blocks with K split over 4 wavefronts
// (op(A) read once for them; with 8 wavefronts they would spill), one tile
// per block with K split over 5 wavefronts, or over 3 wavefronts and 2
// blocks, or 2 wavefronts and 3 blocks (few tiles and long K: the K loop
// of a wavefront waits on memory about once per group of 16 k, so the
// launch is fastest with the shortest loops whose blocks all fit on the
// chip at once; 528 tiles of 8 wavefronts, say, leave 16 blocks for a
// second round at 4 wavefronts per SIMD), for a single
// matrix-vector product the vector-unit kernel, and for a single product of
// at most 32 columns the row-block kernel (zgemm_panel_kernel) with its K
// range split so that 2 or 3 blocks per compute unit hold every block of the
// launch at once.
enum {
  GV_TILE4 = 0,
  GV_SPLIT4,
  GV_SPLIT8,
  GV_WIDE2_S4,
  GV_WIDE4_S4,
  GV_SPLIT5,
  GV_SPLIT3_KB2,
  GV_SPLIT2_KB3,
  GV_GEMV,
  GV_PANEL2,
  GV_PANEL3,
  GV_COUNT
};

static bool single_only(int v) { return v >= GV_WIDE2_S4; }

static bool panel_shape(int v) { return v == GV_PANEL2 || v == GV_PANEL3; }

// compute units of the current device (read once per process)
static int cu_count() {
  static std::atomic<int> n{0};
  int c = n.load();
  if (c == 0) {
    int dev = 0;
    CBFM_HIP(hipGetDevice(&dev));
    CBFM_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    c = std::max(c, 1);
    n.store(c);
  }
  return c;
}

// column blocks per tile and blocks per tile of the launch shapes (the
// row-block shapes: blocks per 64 rows, 2 or 3 blocks per compute unit over
// the launch, at most one per group of 16 k)
static int ct_of(int v) { return v == GV_WIDE4_S4 ? 4 : (v == GV_WIDE2_S4 || panel_shape(v)) ? 2 : 1; }
static int kb_of(int v, int64_t M, int64_t K) {
  if (panel_shape(v)) return panel_blocks_per_rows(M, K, 1, (int64_t)(v == GV_PANEL3 ? 3 : 2) * cu_count());
  return v == GV_SPLIT3_KB2 ? 2 : v == GV_SPLIT2_KB3 ? 3 : 1;
}

// bytes of partial tiles a launch shape leaves for splitk_reduce_kernel
static size_t ws_bytes(int v, int64_t tiles, int64_t M, int64_t N, int64_t K) {
  const int kb = kb_of(v, M, K), ct = ct_of(v);
  if (kb == 1 && !panel_shape(v)) return 0;
  const int64_t t = ct == 1 ? tiles : ((M + 15) / 16) * ((N + 16 * ct - 1) / (16 * ct));
  return (size_t)t * kb * 64 * 8 * ct * sizeof(double);
}

// The row-block kernel takes one product of at most 32 columns with op(A)
// rows and op(B) columns contiguous along k.
static bool panel_fits(int64_t N, int opA, int opB) {
  return N <= 32 && (opA == OP_N || opA == OP_R) && (opB == OP_T || opB == OP_C);
}

// The vector-unit kernel takes one column with op(A) rows contiguous.
static bool gemv_shape(int64_t N, int opA) { return N == 1 && (opA == OP_N || opA == OP_R); }

// tiles: 16 x 16 tiles of the group; M, N, K: the sizes of its product when
// it has one (the wide and row-block shapes number their own tiles)
static void launch_variant(int v, const GemmDesc* dev, int count, int64_t tiles, int64_t M, int64_t N, int64_t K,
                           hipStream_t s, double* ws) {
  const dim3 one((unsigned)tiles);
  auto wide = [&](int ct) { return ((M + 15) / 16) * ((N + 16 * ct - 1) / (16 * ct)); };
  CBFM_REQUIRE(!single_only(v) || count == 1, CBFM_E_ARG, "wide GEMM tiles need a single product");
  switch (v) {
    case GV_GEMV:
      hipLaunchKernelGGL(zgemv_kernel, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, dev);
      break;
    case GV_PANEL2:
    case GV_PANEL3: {
      CBFM_REQUIRE(ws != nullptr, CBFM_E_ARG, "K-split GEMM without workspace");
      CBFM_REQUIRE(N <= 32, CBFM_E_ARG, "row-block GEMM with more than 32 columns");
      const int kb = kb_of(v, M, K);
      const int64_t nt = (M + 15) / 16;
      hipLaunchKernelGGL(zgemm_panel_kernel<2>, dim3((unsigned)((M + 63) / 64 * kb)), dim3(256), 0, s, dev, kb, ws,
                         (int64_t)0, (int64_t)0);
      hipLaunchKernelGGL(panel_reduce_kernel<2>, dim3((unsigned)((nt * 512 + 255) / 256)), dim3(256), 0, s, dev, nt, kb,
                         ws, (int64_t)0);
      break;
    }
    case GV_TILE4:
      hipLaunchKernelGGL((zgemm_batched_kernel<1, 1>), dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, dev, count,
                         tiles);
      break;
    case GV_SPLIT4:
      hipLaunchKernelGGL((zgemm_batched_kernel<4, 1>), one, dim3(256), 0, s, dev, count, tiles);
      break;
    case GV_SPLIT8:
      hipLaunchKernelGGL((zgemm_batched_kernel<8, 1>), one, dim3(512), 0, s, dev, count, tiles);
      break;
    case GV_WIDE2_S4:
      hipLaunchKernelGGL((zgemm_batched_kernel<4, 2>), dim3((unsigned)wide(2)), dim3(256), 0, s, dev, count, wide(2));
      break;
    case GV_SPLIT5:
      hipLaunchKernelGGL((zgemm_batched_kernel<5, 1>), one, dim3(320), 0, s, dev, count, tiles);
      break;
    case GV_SPLIT3_KB2:
      CBFM_REQUIRE(ws != nullptr, CBFM_E_ARG, "K-split GEMM without workspace");
      hipLaunchKernelGGL((zgemm_batched_kernel<3, 1>), dim3((unsigned)(tiles * 2)), dim3(192), 0, s, dev, count, tiles,
                         2, ws);
      hipLaunchKernelGGL(splitk_reduce_kernel<1>, one, dim3(256), 0, s, dev, tiles, 2, ws);
      break;
    case GV_SPLIT2_KB3:
      CBFM_REQUIRE(ws != nullptr, CBFM_E_ARG, "K-split GEMM without workspace");
      hipLaunchKernelGGL((zgemm_batched_kernel<2, 1>), dim3((unsigned)(tiles * 3)), dim3(128), 0, s, dev, count, tiles,
                         3, ws);
      hipLaunchKernelGGL(splitk_reduce_kernel<1>, one, dim3(256), 0, s, dev, tiles, 3, ws);
      break;
    default:
      hipLaunchKernelGGL((zgemm_batched_kernel<4, 4>), dim3((unsigned)wide(4)), dim3(256), 0, s, dev, count, wide(4));
      break;
  }
  CBFM_HIP(hipGetLastError());
}

// Shape class of a group for the tuning cache.
struct GemmKey {
  int dev, count, opA, opB;
  int64_t tiles, M, N, K;
  bool operator<(const GemmKey& o) const {
    return std::tie(dev, count, opA, opB, tiles, M, N, K) < std::tie(o.dev, o.count, o.opA, o.opB, o.tiles, o.M, o.N, o.K);
  }
};

static std::mutex g_tune_mu;
static std::map<GemmKey, int> g_tuned;  // launch shape measured fastest, per shape class

static GemmKey key_of(int dev, const GemmDesc* d, int count, int64_t tiles) {
  int64_t K = 0;
  for (int i = 0; i < count; ++i) K = std::max(K, d[i].K);
  return GemmKey{dev, count, d[0].opA, d[0].opB, tiles, d[0].M, d[0].N, K};
}

// Launch shape v runs a group of this shape class.
static bool applicable(int v, const GemmKey& k) {
  return !(single_only(v) && k.count != 1) && !(v == GV_GEMV && !gemv_shape(k.N, k.opA)) &&
         !(panel_shape(v) && !panel_fits(k.N, k.opA, k.opB));
}

// CBFM_GEMM_SHAPE (for tests and tuning studies): the index of a launch
// shape (the order of the enum above) forced on every group it applies to,
// in place of the tuned or default choice.
static int forced_shape() {
  const char* e = std::getenv("CBFM_GEMM_SHAPE");
  if (e == nullptr || *e == 0) return -1;
  const int v = std::atoi(e);
  return v >= 0 && v < GV_COUNT ? v : -1;
}

// Without a measurement: few tiles get the K split over four wavefronts.
static int choose(const GemmKey& k) {
  const int f = forced_shape();
  if (f >= 0 && applicable(f, k)) return f;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(k);
  if (it != g_tuned.end()) return it->second;
  return k.tiles < 4096 ? GV_SPLIT4 : GV_TILE4;
}

static void launch_descs(const GemmDesc* dev, int count, int64_t tiles, int64_t M, int64_t N, int64_t K,
                         double flops, int variant, hipStream_t s, double* ws) {
  TimedLaunch tl(T_GEMM, s, flops);
  if (panel_shape(variant)) {
    TimedLaunch tp(T_GEMM_PANEL, s, flops);
    launch_variant(variant, dev, count, tiles, M, N, K, s, ws);
  } else {
    launch_variant(variant, dev, count, tiles, M, N, K, s, ws);
  }
}

// Elements spanned by an operand or the result of a descriptor.
static int64_t extent(int64_t rows, int64_t cols, int64_t ld) { return (rows - 1) * ld + cols; }

// A group may be run repeatedly for timing only if every product overwrites
// its result without reading it and no result overlaps an operand.
static bool rerunnable(const std::vector<GemmDesc>& g) {
  for (const GemmDesc& d : g) {
    if (d.accumulate) return false;
    const char* c0 = reinterpret_cast<const char*>(d.C);
    const char* c1 = c0 + 16 * (d.transC ? extent(d.N, d.M, d.ldc) : extent(d.M, d.N, d.ldc));
    for (const GemmDesc& e : g) {
      const bool ta = e.opA == OP_T || e.opA == OP_C, tb = e.opB == OP_T || e.opB == OP_C;
      const char* a0 = reinterpret_cast<const char*>(e.A);
      const char* a1 = a0 + 16 * (ta ? extent(e.K, e.M, e.lda) : extent(e.M, e.K, e.lda));
      const char* b0 = reinterpret_cast<const char*>(e.B);
      const char* b1 = b0 + 16 * (tb ? extent(e.N, e.K, e.ldb) : extent(e.K, e.N, e.ldb));
      if ((c0 < a1 && a0 < c1) || (c0 < b1 && b0 < c1)) return false;
    }
  }
  return true;
}

// Autotuning: time every launch shape on the group itself (one warm-up and
// three timed launches each) and remember the fastest for its shape class.
static void tune_group(const GemmKey& key, const GemmDesc* dev, int count, int64_t tiles, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tuned.count(key)) return;
  }
  hipEvent_t e0, e1;
  CBFM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw Error{CBFM_E_HIP, "hipEventCreate failed"};
  }
  int best = choose(key);
  float best_ms = 0;
  try {
    size_t wsb = 0;
    if (count == 1)
      for (int v = 0; v < GV_COUNT; ++v) wsb = std::max(wsb, ws_bytes(v, tiles, key.M, key.N, key.K));
    Scratch ws(wsb, s);
    for (int v = 0; v < GV_COUNT; ++v) {
      if (!applicable(v, key)) continue;
      launch_variant(v, dev, count, tiles, key.M, key.N, key.K, s, ws.as<double>());
      CBFM_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) launch_variant(v, dev, count, tiles, key.M, key.N, key.K, s, ws.as<double>());
      CBFM_HIP(hipEventRecord(e1, s));
      CBFM_HIP(hipEventSynchronize(e1));
      float ms = 0;
      CBFM_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (v == 0 || ms < best_ms) {
        best = v;
        best_ms = ms;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
}

void zgemm_batched(std::vector<GemmDesc>& descs, hipStream_t s, std::vector<std::vector<GemmDesc>>* keep) {
  if (descs.empty()) return;
  std::vector<GemmDesc> live;
  double flops = 0;
  const int64_t tiles = number_tiles(descs, live, &flops);
  if (live.empty()) return;
  Scratch dev(live.size() * sizeof(GemmDesc), s);
  CBFM_HIP(hipMemcpyAsync(dev.p, live.data(), live.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
  int d = 0;
  CBFM_HIP(hipGetDevice(&d));
  const GemmKey key = key_of(d, live.data(), (int)live.size(), tiles);
  const int v = choose(key);
  Scratch ws(ws_bytes(v, tiles, key.M, key.N, key.K), s);
  launch_descs(dev.as<GemmDesc>(), (int)live.size(), tiles, key.M, key.N, key.K, flops, v, s, ws.as<double>());
  if (keep) {  // the caller keeps the staged descriptors until it synchronises s
    keep->push_back(std::move(live));
    return;
  }
  // the descriptor staging buffer is host memory of this frame
  CBFM_HIP(hipStreamSynchronize(s));
}

// Row-block kernel launches of nb products (see gemm.h): 16 columns per
// tile up to N = 16, else 32; as many blocks as fit on the chip at once
// (4 per compute unit with 16 columns, 3 with 32).
static int panel_ct(int64_t N) { return N <= 16 ? 1 : 2; }
static int panel_batch_kb(const GemmDesc& d, int64_t nb) {
  return panel_blocks_per_rows(d.M, d.K, nb, (int64_t)(panel_ct(d.N) == 1 ? 4 : 3) * cu_count());
}

size_t panel_batch_ws_bytes(const GemmDesc& d, int64_t nb) {
  const int ct = panel_ct(d.N);
  return (size_t)nb * ((d.M + 15) / 16) * panel_batch_kb(d, nb) * 64 * 8 * ct * sizeof(double);
}

void panel_batch(const GemmDesc* dev, const GemmDesc& d, int64_t nb, int64_t sA, int64_t sB, int64_t sC, double* ws,
                 hipStream_t s) {
  CBFM_REQUIRE(nb >= 1 && d.M >= 1 && d.N >= 1 && d.K >= 0 && panel_fits(d.N, d.opA, d.opB), CBFM_E_ARG,
               "row-block GEMM: one to 32 columns, op(A) rows and op(B) columns contiguous along k");
  CBFM_REQUIRE(ws != nullptr, CBFM_E_ARG, "K-split GEMM without workspace");
  const int kb = panel_batch_kb(d, nb);
  const int64_t nt = nb * ((d.M + 15) / 16), blocks = nb * ((d.M + 63) / 64) * kb;
  if (panel_ct(d.N) == 1) {
    hipLaunchKernelGGL(zgemm_panel_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, dev, kb, ws, sA, sB);
    hipLaunchKernelGGL(panel_reduce_kernel<1>, dim3((unsigned)((nt * 256 + 255) / 256)), dim3(256), 0, s, dev, nt, kb,
                       ws, sC);
  } else {
    hipLaunchKernelGGL(zgemm_panel_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, dev, kb, ws, sA, sB);
    hipLaunchKernelGGL(panel_reduce_kernel<2>, dim3((unsigned)((nt * 512 + 255) / 256)), dim3(256), 0, s, dev, nt, kb,
                       ws, sC);
  }
  CBFM_HIP(hipGetLastError());
}

GemmPlan::GemmPlan(const std::vector<std::vector<GemmDesc>>& groups, hipStream_t s, bool tune)
    : tune_(tune), dev_(std::max<size_t>(1, [&] {
             size_t k = 0;
             for (const auto& g : groups) k += g.size();
             return k;
           }()) * sizeof(GemmDesc),
           s) {
  std::vector<GemmDesc> all;
  for (const auto& g : groups) {
    first_.push_back((int64_t)all.size());
    double f = 0;
    tiles_.push_back(number_tiles(g, all, &f));
    flops_.push_back(f);
    count_.push_back((int64_t)all.size() - first_.back());
  }
  if (!all.empty()) {
    CBFM_HIP(hipMemcpyAsync(dev_.p, all.data(), all.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
    CBFM_HIP(hipStreamSynchronize(s));  // `all` is host memory of this frame
  }
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  GemmKey last{-1, 0, 0, 0, 0, 0, 0, 0};  // groups of one shape class (such as the
  int last_variant = GV_TILE4;             // per-Krylov-index matvecs) share one choice
  for (size_t g = 0; g < groups.size(); ++g) {
    m_.push_back(count_[g] > 0 ? all[first_[g]].M : 0);
    n_.push_back(count_[g] > 0 ? all[first_[g]].N : 0);
    int64_t kmax = 0;
    for (int64_t i = 0; i < count_[g]; ++i) kmax = std::max(kmax, all[first_[g] + i].K);
    k_.push_back(kmax);
    if (count_[g] == 0) {
      variant_.push_back(GV_TILE4);
      continue;
    }
    const GemmKey k = key_of(dev, all.data() + first_[g], (int)count_[g], tiles_[g]);
    if (last.dev >= 0 && !(k < last) && !(last < k)) {
      variant_.push_back(last_variant);
      continue;
    }
    if (tune_ && rerunnable(groups[g])) tune_group(k, dev_.as<GemmDesc>() + first_[g], (int)count_[g], tiles_[g], s);
    last = k;
    last_variant = choose(k);
    variant_.push_back(last_variant);
  }
  // one workspace for the partial tiles of every group (launched in turn)
  size_t wsb = 0;
  for (size_t g = 0; g < groups.size(); ++g)
    wsb = std::max(wsb, ws_bytes(variant_[g], tiles_[g], m_[g], n_[g], k_[g]));
  ws_.reset(new Scratch(wsb, s));
}

void GemmPlan::launch(size_t g, hipStream_t s) const {
  CBFM_REQUIRE(g < tiles_.size(), CBFM_E_ARG, "GEMM plan group out of range");
  if (count_[g] == 0) return;
  launch_descs(dev_.as<GemmDesc>() + first_[g], (int)count_[g], tiles_[g], m_[g], n_[g], k_[g], flops_[g],
               variant_[g], s, ws_->as<double>());
}

}  // namespace cbfm
