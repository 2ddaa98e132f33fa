// Internal structures of libcbfm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cbfm.h"

namespace cbfm {

void set_error(const std::string& msg);

struct Error {
  cbfm_status code;
  std::string msg;
};

#define CBFM_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::cbfm::Error{CBFM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define CBFM_REQUIRE(cond, code, msg)                 \
  do {                                                \
    if (!(cond)) throw ::cbfm::Error{code, (msg)};    \
  } while (0)

// Run a body, translating exceptions into a status.
template <typename F>
cbfm_status guarded(F&& f) {
  try {
    f();
    return CBFM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return CBFM_E_NOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return CBFM_E_HIP;
  }
}

// Device memory of the library: from the caller's allocator when one is
// set (cbfm_set_allocator), else from hipMalloc.  A block remembers the
// release routine it must go back through.
using ReleaseFn = void (*)(void* p, void* stream);
// device bytes the library holds from hipMalloc (handles and the scratch
// cache), now and at most since the process started
void device_bytes_add(int64_t delta);
// the caller's allocator, or nullptr (then hipMalloc)
void* hooked_alloc(size_t bytes, hipStream_t s, ReleaseFn* release);

// Device buffer owned by a handle.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ReleaseFn rel = nullptr;  // the caller's release routine, or nullptr (hipFree)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    ReleaseFn r = nullptr;
    void* q = hooked_alloc(n, nullptr, &r);
    if (r) {
      CBFM_REQUIRE(q != nullptr, CBFM_E_NOMEM, "the caller's allocator returned no memory for " + std::to_string(n) + " bytes");
      p = q;
      rel = r;
      bytes = n;
      return;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{CBFM_E_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
    device_bytes_add((int64_t)n);
  }
  template <typename T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) CBFM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  void release() {
    if (p && rel) {
      rel(p, nullptr);
    } else if (p) {
      (void)hipFree(p);
      device_bytes_add(-(int64_t)bytes);
    }
    p = nullptr;
    bytes = 0;
    rel = nullptr;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Scratch allocation (scratch.cpp): device blocks kept after use and handed
// out again, reuse ordered on the stream by an event; blocks from
// kBigScratch up are matched by size rather than by power-of-two class.
constexpr size_t kBigScratch = (size_t)256 << 20;
// *block receives the size of the block handed out (at least `bytes`; a
// cached block may be larger), which scratch_release must be given back.
void* scratch_alloc(size_t bytes, hipStream_t s, size_t* block);
void scratch_release(void* p, size_t block, hipStream_t s);
size_t scratch_cached_bytes();  // bytes held by the cache on the current device
// Before destroying stream s: synchronise it, then call this, so that the
// cache drops every reference to s and to the events recorded on it.
void scratch_forget_stream(hipStream_t s);
// Marks s as a library side stream: a cached block it released and still
// uses is not waited for by another stream while a new block can be had.
void scratch_side_stream(hipStream_t s);
// Frees the oldest cached blocks of the current device (after their events
// complete) until the cache holds at most `limit` bytes.
void scratch_trim_to(size_t limit);

// Stream-ordered scratch released at scope exit: from the caller's
// allocator when one is set, else from the library's cache.
struct Scratch {
  void* p = nullptr;
  hipStream_t s = nullptr;
  size_t n = 0;      // bytes asked for
  size_t block = 0;  // size of the cache block behind p
  ReleaseFn rel = nullptr;
  Scratch(size_t bytes, hipStream_t stream) : s(stream), n(bytes) {
    if (bytes == 0) return;
    p = hooked_alloc(bytes, stream, &rel);
    if (rel) {
      CBFM_REQUIRE(p != nullptr, CBFM_E_NOMEM,
                   "the caller's allocator returned no memory for " + std::to_string(bytes) + " bytes");
      return;
    }
    p = scratch_alloc(bytes, stream, &block);
  }
  ~Scratch() {
    if (p && rel)
      rel(p, s);
    else if (p)
      scratch_release(p, block, s);
  }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Per-triangle geometry, structure of arrays, in one precision.  Points are
// stored relative to the triangle's centroid; the centroid itself is kept
// in double for both precisions (pair offsets are formed in double).
template <typename R>
struct TriTab {
  const R* q[3];    // quadrature points, [k * nt + t], k < 7
  const R* v[3];    // vertices (free vertices of the local functions), [a * nt + t]
  const R* c;       // s_a * l_a, [a * nt + t]
  const double* cen[3];  // centroid
  int64_t nt;
};

struct NearPair {
  int32_t p, q;     // triangles
  int32_t i, j;     // positions in the row / column triangle lists
  int32_t coplanar; // K of the pair is zero
  int32_t pad;      // batched near-pair launches: the block the pair belongs to
};

struct MeshHost {
  int64_t nv = 0, nt = 0, ne = 0;
  int32_t nblocks = 1;
  std::vector<double> V;            // nv*3
  std::vector<int32_t> T;           // nt*3
  std::vector<int32_t> edges;       // ne*2 canonical
  std::vector<int32_t> tplus, tminus, aplus, aminus;
  std::vector<int32_t> tri_edge;    // nt*3
  std::vector<int32_t> tri_sign;    // nt*3
  std::vector<double> length;       // ne
  std::vector<double> area;         // nt
  std::vector<double> normal;       // nt*3
  std::vector<double> centroid;     // nt*3
  std::vector<int32_t> edge_block;  // ne
  std::vector<int32_t> perm;        // internal (cell-sorted) -> canonical
  std::vector<int32_t> iperm;       // canonical -> internal
  std::vector<int64_t> cell_off;    // nblocks+1 offsets into the internal order
  std::vector<NearPair> near;       // all near pairs (i = p, j = q)
};

}  // namespace cbfm

struct cbfm_mesh_s {
  cbfm::MeshHost h;
  // every cell a translated copy of cell 0 (the same RWGs in the same order
  // on triangles shifted by shift[b]), with no triangle carrying RWGs of
  // two cells; found at load (find_translates in mesh.cpp)
  bool translated = false;
  std::vector<double> shift;   // nblocks * 3
  std::vector<int32_t> tcell;  // triangle -> its cell (translated meshes)
  // device tables
  cbfm::DevBuf q64, v64, c64, q32, v32, c32, cen;   // SoA geometry
  cbfm::DevBuf tri_edge, tri_sign, tplus, tminus, aplus, aminus, length, area;
  cbfm::DevBuf tri_xyz;        // nt*9 absolute vertex coordinates (double)
  cbfm::DevBuf perm, iperm;    // int32
  cbfm::TriTab<double> tab64() const;
  cbfm::TriTab<float> tab32() const;
};

namespace cbfm {

// Opt-in launch timing (see cbfm_timer_enable): start/stop bracket one
// launch of kernel family `id` on stream s, with its algorithmic work (the
// family's unit: triangle pairs, real flops or bytes); no-ops when timing
// is off.
enum TimerId {
  T_FILL_REGULAR = 0,
  T_FILL_NEAR = 1,
  T_ASSEMBLE = 2,
  T_GEMM = 3,
  T_GMRES_DOTS = 4,
  T_GMRES_UPDATE = 5,
  T_FILL_REGULAR_F32 = 6,  // the regular fill in float
  T_XGEMM = 7,             // GEMMs on the FP32 / BF16 matrix cores
  T_GEMM_PANEL = 8,        // the T_GEMM launches run by the row-block kernel
  T_COUNT = 9
};
struct TimedLaunch {
  TimedLaunch(int id, hipStream_t s, double work = 0.0);
  ~TimedLaunch();
  int id;
  hipStream_t s;
  double work;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

struct Media {
  // exterior k1 real; interior k2 = k2r + j k2i (k2i <= 0 when lossy)
  double k1, k2r, k2i;
  std::complex<double> eta1, eta2;
};

Media make_media(const cbfm_medium* med);

// Fill the triangle-local matrix for row triangles x column triangles into
// `local` (3 ops x 3*nrt x 3*nct complex of the given precision, ops per
// layout) and overwrite the near pairs.  Implemented in fill.hip.
// One regular fill of many (mesh, medium, rows x columns) jobs in a single
// persistent launch (the near pairs of each job are left to fill_near).
struct FillBatchItem {
  const cbfm_mesh_s* m;
  Media md;
  int layout;
  const int32_t* rowTris;
  int64_t nrt;
  const int32_t* colTris;
  int64_t nct;
  void* local;
};
void fill_regular_batch(const std::vector<FillBatchItem>& items, int precision, hipStream_t s);
// transposed: pair (p, q) is written into the slot of (q, p) (row i, column
// j), each 3 x 3 block transposed, as the reversed pair's entries.
void fill_near(const cbfm_mesh_s* m, const Media& md, int precision, int layout, const NearPair* near, int64_t nnear,
               int64_t nrt, int64_t nct, void* local, hipStream_t s, int transposed = 0);
// The near pairs of several FP64 local blocks in one launch pair: pair t
// (device arrays) writes into block outs[near[t].pad - cell0], which starts
// outs[...].off elements into `local`.
struct NearOut {
  int64_t off, op_stride, ldl;
};
void fill_near_batch(const cbfm_mesh_s* m, const Media& md, int layout, const NearPair* near, int64_t nnear,
                     const NearOut* outs, int cell0, void* local, hipStream_t s);
// near_buf: near_buffer_bytes(nnear) bytes of device memory for the near
// stage's intermediates, or NULL for stream-ordered scratch.
void fill_local(const cbfm_mesh_s* m, const Media& md, int precision, int layout,
                const int32_t* rowTris_dev, int64_t nrt, const int32_t* colTris_dev, int64_t nct,
                const NearPair* near_dev, int64_t nnear, void* local, hipStream_t s, void* near_buf = nullptr);
size_t near_buffer_bytes(int64_t nnear);

void rhs_launch(const cbfm_mesh_s* m, const Media& md, double eta0, const double* inc_dev, int64_t nrhs,
                void* v_dev, hipStream_t s);

// Gather the RWG matrices [op][r][c] (r < nrow, c < ncol) of the listed
// canonical edges from a triangle-local buffer.  With precision FP32 the
// local buffer holds float2 and Z receives double2 when out_fp64 is set.
void assemble(const cbfm_mesh_s* m, int precision, const void* local, int64_t nrt, int64_t nct,
              const int32_t* rowEdges, int64_t nrow, const int32_t* colEdges, int64_t ncol,
              const int32_t* rowPos, const int32_t* colPos, void* Z, int64_t zop_stride, int64_t ldz,
              hipStream_t s, int out_fp64 = 0);
// The same for the RWG pairs listed in pairs (npairs (row, column) index
// pairs into rowEdges and colEdges), into Z[op][row][column].
void assemble_pairs(const cbfm_mesh_s* m, int precision, const void* local, int64_t nrt, int64_t nct,
                    const int32_t* rowEdges, const int32_t* colEdges, const int32_t* pairs, int64_t npairs,
                    const int32_t* rowPos, const int32_t* colPos, void* Z, int64_t zop_stride, int64_t ldz,
                    hipStream_t s, int out_fp64 = 0);

}  // namespace cbfm
