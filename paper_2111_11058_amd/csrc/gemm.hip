// Batched, variable-size complex double GEMM on the gfx950 matrix cores:
//   C = alpha * op(A) * op(B) (+ C if accumulate)
// op in {N, T (transpose), C (conjugate transpose), R (conjugate)}, all
// matrices row-major complex double with leading dimensions.
//
// A wavefront computes a 16 x 16 tile of C with v_mfma_f64_16x16x4_f64
// (real): for each group of 16 k it does 4 x 4 MFMAs, the four real
// products Ar*Br, -Ai*Bi, Ar*Bi, Ai*Br.  Lane L holds A[L % 16][k] and
// B[k][L % 16] for k = k0 + 4 (L / 16) + t, t = 0..3 (any assignment of the
// 16 k values to (slot, step) works as long as A and B agree), which lets
// each lane load 4 consecutive elements when op(A) is not transposed.
// The accumulator element r of lane L is C[4 r + L / 16][L % 16] (measured
// on gfx950 with indexed operands: rows are interleaved across the four
// lane groups).
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"
#include "gemm.h"

namespace cbfm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 ld_op(const double2* __restrict__ X, int64_t ld, int op, int64_t i, int64_t k,
                                         int64_t rows, int64_t cols) {
  // element op(X)[i][k]; rows x cols is the shape of op(X); zero outside.
  // Branch-free: an out-of-range lane loads element (0, 0) and discards it.
  const bool ok = i < rows && k < cols;
  const int64_t ii = ok ? i : 0, kk = ok ? k : 0;
  const int64_t idx = (op == OP_N || op == OP_R) ? ii * ld + kk : kk * ld + ii;
  double2 v = X[idx];
  v.x = ok ? v.x : 0.0;
  v.y = ok ? ((op == OP_C || op == OP_R) ? -v.y : v.y) : 0.0;
  return v;
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(x & 0xffffffff));
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// SPLITK = 1: each of the 4 wavefronts of a block owns a tile.
// SPLITK > 1: the SPLITK wavefronts of a block share one tile, each taking
// every SPLITK-th group of 16 k, and the partial tiles are summed through
// LDS (few, deep tiles: more loads in flight per tile).
template <int SPLITK>
__global__ void __launch_bounds__(SPLITK == 1 ? 256 : 64 * SPLITK)
    zgemm_batched_kernel(const GemmDesc* __restrict__ desc, int ndesc, int64_t total_tiles) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // wave-uniform tile and descriptor (readfirstlane makes the K loop a scalar
  // loop: the accumulators then stay in the matrix-core registers across it)
  const int64_t tile = SPLITK == 1 ? (int64_t)blockIdx.x * 4 + wave : (int64_t)blockIdx.x;
  __shared__ double red[SPLITK == 1 ? 1 : (SPLITK - 1) * 64 * 8];
  if (tile >= total_tiles) return;  // uniform per block when SPLITK == 4
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
  const int64_t t = tile - d.tile_start;
  const int64_t ntn = (d.N + 15) / 16;
  const int64_t m0 = (t / ntn) * 16, n0 = (t % ntn) * 16;
  const int64_t ia = m0 + (lane & 15);  // row of op(A) this lane loads
  const int64_t jb = n0 + (lane & 15);  // column of op(B) this lane loads
  const int slot = lane >> 4;
  dbl4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  const int64_t kstep = 16 * SPLITK;
  int64_t k0 = SPLITK == 1 ? 0 : 16 * wave;
  double2 a[4], b[4];
  if (k0 < d.K) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * slot + s;
      a[s] = ld_op(d.A, d.lda, d.opA, ia, k, d.M, d.K);
      b[s] = ld_op(d.B, d.ldb, d.opB, k, jb, d.K, d.N);
    }
  }
  for (; k0 < d.K; k0 += kstep) {
    // prefetch the next group while the matrix cores work on this one
    double2 an[4], bn[4];
    const int64_t k1 = k0 + kstep;
    if (k1 < d.K) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t k = k1 + 4 * slot + s;
        an[s] = ld_op(d.A, d.lda, d.opA, ia, k, d.M, d.K);
        bn[s] = ld_op(d.B, d.ldb, d.opB, k, jb, d.K, d.N);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].x, b[s].x, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[s].y, b[s].y, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].x, b[s].y, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].y, b[s].x, ci, 0, 0, 0);
    }
    if (k1 < d.K) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a[s] = an[s];
        b[s] = bn[s];
      }
    }
  }
  if (SPLITK > 1) {
    // waves 1..SPLITK-1 hand their partial tiles to wave 0
    if (wave > 0) {
      double* r = red + ((wave - 1) * 64 + lane) * 8;
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
      const double* r = red + (w * 64 + lane) * 8;
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
    const int64_t row = m0 + 4 * r + slot;
    if (row < d.M) {
      const double xr = cr[r], xi = ci[r];
      double2 v = make_double2(d.alpha_re * xr - d.alpha_im * xi, d.alpha_re * xi + d.alpha_im * xr);
      double2* p = d.transC ? d.C + col * d.ldc + row : d.C + row * d.ldc + col;
      if (d.accumulate) {
        const double2 o = *p;
        v.x += o.x;
        v.y += o.y;
      }
      *p = v;
    }
  }
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

__device__ __forceinline__ float2 ldx(const void* __restrict__ X, int is64, int64_t ld, int op, int64_t i, int64_t k,
                                      int64_t rows, int64_t cols) {
  const bool ok = i < rows && k < cols;
  const int64_t ii = ok ? i : 0, kk = ok ? k : 0;
  const int64_t idx = (op == OP_N || op == OP_R) ? ii * ld + kk : kk * ld + ii;
  float2 v;
  if (is64) {
    const double2 d = static_cast<const double2*>(X)[idx];
    v = make_float2((float)d.x, (float)d.y);
  } else {
    v = static_cast<const float2*>(X)[idx];
  }
  v.x = ok ? v.x : 0.0f;
  v.y = ok ? ((op == OP_C || op == OP_R) ? -v.y : v.y) : 0.0f;
  return v;
}

template <int MODE, int SPLITK>
__global__ void __launch_bounds__(256) xgemm_batched_kernel(const GemmDescX* __restrict__ desc, int ndesc,
                                                            int64_t total_tiles) {
  constexpr int KG = MODE == XG_FP32 ? 16 : 32;  // k per step of a wavefront
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tile = SPLITK == 1 ? (int64_t)blockIdx.x * 4 + wave : (int64_t)blockIdx.x;
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
  d.a64 = __builtin_amdgcn_readfirstlane(d.a64);
  d.b64 = __builtin_amdgcn_readfirstlane(d.b64);
  const int64_t t = tile - d.tile_start;
  const int64_t ntn = (d.N + 15) / 16;
  const int64_t m0 = (t / ntn) * 16, n0 = (t % ntn) * 16;
  const int64_t ia = m0 + (lane & 15), jb = n0 + (lane & 15);
  const int slot = lane >> 4;
  flt4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  for (int64_t k0 = SPLITK == 1 ? 0 : (int64_t)KG * wave; k0 < d.K; k0 += (int64_t)KG * SPLITK) {
    if constexpr (MODE == XG_FP32) {
      float2 a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t k = k0 + 4 * slot + q;
        a[q] = ldx(d.A, d.a64, d.lda, d.opA, ia, k, d.M, d.K);
        b[q] = ldx(d.B, d.b64, d.ldb, d.opB, k, jb, d.K, d.N);
      }
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
      for (int q = 0; q < 8; ++q) {
        const int64_t k = k0 + 8 * slot + q;
        const float2 a = ldx(d.A, d.a64, d.lda, d.opA, ia, k, d.M, d.K);
        const float2 b = ldx(d.B, d.b64, d.ldb, d.opB, k, jb, d.K, d.N);
        ar[q] = (__bf16)a.x;
        ai[q] = (__bf16)a.y;
        an[q] = (__bf16)(-a.y);
        br[q] = (__bf16)b.x;
        bi[q] = (__bf16)b.y;
      }
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
        const int64_t k = k0 + 8 * slot + q;
        const float2 a = ldx(d.A, d.a64, d.lda, d.opA, ia, k, d.M, d.K);
        const float2 b = ldx(d.B, d.b64, d.ldb, d.opB, k, jb, d.K, d.N);
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

static void launch_x(const GemmDescX* dd, int n, int64_t tiles, double flops, int mode, hipStream_t s) {
  TimedLaunch tl(T_GEMM, s, flops);
  const bool few = tiles < 4096;
  const dim3 g(few ? (unsigned)tiles : (unsigned)((tiles + 3) / 4));
  if (mode == XG_BF16) {
    if (few)
      hipLaunchKernelGGL((xgemm_batched_kernel<XG_BF16, 4>), g, dim3(256), 0, s, dd, n, tiles);
    else
      hipLaunchKernelGGL((xgemm_batched_kernel<XG_BF16, 1>), g, dim3(256), 0, s, dd, n, tiles);
  } else if (mode == XG_BF16X3) {
    if (few)
      hipLaunchKernelGGL((xgemm_batched_kernel<XG_BF16X3, 4>), g, dim3(256), 0, s, dd, n, tiles);
    else
      hipLaunchKernelGGL((xgemm_batched_kernel<XG_BF16X3, 1>), g, dim3(256), 0, s, dd, n, tiles);
  } else {
    if (few)
      hipLaunchKernelGGL((xgemm_batched_kernel<XG_FP32, 4>), g, dim3(256), 0, s, dd, n, tiles);
    else
      hipLaunchKernelGGL((xgemm_batched_kernel<XG_FP32, 1>), g, dim3(256), 0, s, dd, n, tiles);
  }
  CBFM_HIP(hipGetLastError());
}

void xgemm_batched(std::vector<GemmDescX>& descs, int mode, hipStream_t s) {
  if (descs.empty()) return;
  std::vector<GemmDescX> live;
  double flops = 0;
  const int64_t tiles = number_tiles_x(descs, live, &flops);
  if (live.empty()) return;
  Scratch dev(live.size() * sizeof(GemmDescX), s);
  CBFM_HIP(hipMemcpyAsync(dev.p, live.data(), live.size() * sizeof(GemmDescX), hipMemcpyHostToDevice, s));
  launch_x(dev.as<GemmDescX>(), (int)live.size(), tiles, flops, mode, s);
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
  }
  if (!all.empty()) {
    CBFM_HIP(hipMemcpyAsync(dev_.p, all.data(), all.size() * sizeof(GemmDescX), hipMemcpyHostToDevice, s));
    CBFM_HIP(hipStreamSynchronize(s));  // `all` is host memory of this frame
  }
}

void XGemmPlan::launch(size_t g, hipStream_t s) const {
  CBFM_REQUIRE(g < tiles_.size(), CBFM_E_ARG, "GEMM plan group out of range");
  if (count_[g] == 0) return;
  launch_x(dev_.as<GemmDescX>() + first_[g], (int)count_[g], tiles_[g], flops_[g], mode_, s);
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

// Launch shapes: four tiles per block (one per wavefront), or one tile per
// block with K split over 4 or 8 wavefronts (16 would need more registers
// than a 1024-thread block leaves a lane).
enum { GV_TILE4 = 0, GV_SPLIT4, GV_SPLIT8, GV_COUNT };

static void launch_variant(int v, const GemmDesc* dev, int count, int64_t tiles, hipStream_t s) {
  const dim3 one((unsigned)tiles);
  switch (v) {
    case GV_TILE4:
      hipLaunchKernelGGL(zgemm_batched_kernel<1>, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, dev, count,
                         tiles);
      break;
    case GV_SPLIT4:
      hipLaunchKernelGGL(zgemm_batched_kernel<4>, one, dim3(256), 0, s, dev, count, tiles);
      break;
    default:
      hipLaunchKernelGGL(zgemm_batched_kernel<8>, one, dim3(512), 0, s, dev, count, tiles);
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

static GemmKey key_of(const GemmDesc* d, int count, int64_t tiles) {
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  int64_t K = 0;
  for (int i = 0; i < count; ++i) K = std::max(K, d[i].K);
  return GemmKey{dev, count, d[0].opA, d[0].opB, tiles, d[0].M, d[0].N, K};
}

// Without a measurement: few tiles get the K split over four wavefronts.
static int choose(const GemmKey& k) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(k);
  if (it != g_tuned.end()) return it->second;
  return k.tiles < 4096 ? GV_SPLIT4 : GV_TILE4;
}

static void launch_descs(const GemmDesc* dev, int count, int64_t tiles, double flops, int variant, hipStream_t s) {
  TimedLaunch tl(T_GEMM, s, flops);
  launch_variant(variant, dev, count, tiles, s);
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
    for (int v = 0; v < GV_COUNT; ++v) {
      launch_variant(v, dev, count, tiles, s);
      CBFM_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) launch_variant(v, dev, count, tiles, s);
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

void zgemm_batched(std::vector<GemmDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  std::vector<GemmDesc> live;
  double flops = 0;
  const int64_t tiles = number_tiles(descs, live, &flops);
  if (live.empty()) return;
  Scratch dev(live.size() * sizeof(GemmDesc), s);
  CBFM_HIP(hipMemcpyAsync(dev.p, live.data(), live.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
  launch_descs(dev.as<GemmDesc>(), (int)live.size(), tiles, flops, choose(key_of(live.data(), (int)live.size(), tiles)),
               s);
  // the descriptor staging buffer is host memory of this frame
  CBFM_HIP(hipStreamSynchronize(s));
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
  for (size_t g = 0; g < groups.size(); ++g) {
    if (count_[g] == 0) {
      variant_.push_back(GV_TILE4);
      continue;
    }
    const GemmKey k = key_of(all.data() + first_[g], (int)count_[g], tiles_[g]);
    if (tune_ && rerunnable(groups[g])) tune_group(k, dev_.as<GemmDesc>() + first_[g], (int)count_[g], tiles_[g], s);
    variant_.push_back(choose(k));
  }
}

void GemmPlan::launch(size_t g, hipStream_t s) const {
  CBFM_REQUIRE(g < tiles_.size(), CBFM_E_ARG, "GEMM plan group out of range");
  if (count_[g] == 0) return;
  launch_descs(dev_.as<GemmDesc>() + first_[g], (int)count_[g], tiles_[g], flops_[g], variant_[g], s);
}

}  // namespace cbfm
