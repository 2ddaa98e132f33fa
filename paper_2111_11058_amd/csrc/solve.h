// The device GMRES engine (solve.hip) shared by the reduced CBFM solve, the
// full-system (MoM) solve, the IPCBF generation and the matrix-free
// reduced operator.
#pragma once

#include <vector>

#include "internal.h"

namespace cbfm {

// A linear operator on vectors of length n, applied to nrhs vectors at once
// (vector after vector).  Dense operators expose their matrix (row-major,
// double and/or float); composite ones implement prepare/launch/apply.
class KrylovOp {
 public:
  virtual ~KrylovOp() = default;
  virtual const double2* dense64(int64_t* lda) const {
    (void)lda;
    return nullptr;
  }
  virtual const float2* dense32(int64_t* lda) const {
    (void)lda;
    return nullptr;
  }
  // composite operators (double Krylov basis only): once the basis V
  // (basis index j, vector c at V + j vstride + c n) and the product w are
  // allocated, prepare the products w = A q_j for j < mres
  virtual void prepare(const double2* V, int64_t vstride, double2* w, int64_t mres, int64_t nrhs, hipStream_t s) {
    (void)V, (void)vstride, (void)w, (void)mres, (void)nrhs, (void)s;
  }
  virtual void launch(int64_t j, hipStream_t q) const { (void)j, (void)q; }
  // r = A x for nrhs vectors (double)
  virtual void apply(const double2* x, double2* r, int64_t nrhs, hipStream_t s) const {
    (void)x, (void)r, (void)nrhs, (void)s;
  }
  // flexible GMRES: the basis the iterate is built from (z_j = M_j^{-1} q_j,
  // same layout as the Krylov basis), or nullptr for the Krylov basis itself
  virtual const double2* xbasis() const { return nullptr; }
};

struct GmresSpec {
  double tol = 1e-6;
  int64_t max_iter = 1000, restart = 100;
  bool f32 = false;        // float Krylov basis, cycles refined against the double residual
  double inner_tol = 0.0;  // f32 only: relative reduction per cycle (0: 1e-6)
  bool graph = false;      // Arnoldi chunks replayed from a HIP graph (dense operators)
  bool basis32 = false;    // double cycles with the Krylov basis stored in float (dense double
                           // operator); each cycle stops at a reduction of inner_tol as in f32
  int sstep = 0;           // 4 or 8: s-step cycles of blocks of that many iterations (dense double
                           // operator, double basis, no graphs); 0: plain cycles
  int block = 0;           // block GMRES: the right-hand sides share one Krylov space per group
                           // (1: groups of up to 32 sized for cycles of 32 block iterations or more;
                           // 2..32: groups of that many); dense double or float operator (a float
                           // one only with f32 unset), double basis, no graphs; restart and
                           // max_iter then count block iterations
};

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

struct GmresResult {
  std::vector<int32_t> its;
  std::vector<double> res;  // true relative residual ||b - A x|| / ||b|| at the end
  bool noconv = false;      // some res > tol
};

// Right-hand sides b and iterate x: nrhs x n double, device (x starts at 0).
GmresResult gmres_run(KrylovOp& op, int64_t n, int64_t nrhs, const double2* b, double2* x, const GmresSpec& p,
                      hipStream_t s);

// Block GMRES (bgmres.hip) on a dense operator, double (A) or, when A is
// null, float (A32: its products on the FP32 matrix cores, the Krylov basis
// and everything else in double, so the Arnoldi relation holds to float
// rounding): b, x as gmres_run; the iteration counts returned are block
// iterations.
GmresResult block_gmres_run(const double2* A, int64_t lda, const float2* A32, int64_t lda32, int64_t n, int64_t nrhs,
                            const double2* b, double2* x, const GmresSpec& p, hipStream_t s);

// Dense row-major operator: the double matrix (lda), the float one (n), or
// both (a float-only operator forms its residuals in float too).
class DenseOp : public KrylovOp {
 public:
  DenseOp(const double2* A64, int64_t lda, const float2* A32, int64_t lda32)
      : A64_(A64), lda_(lda), A32_(A32), lda32_(lda32) {}
  const double2* dense64(int64_t* lda) const override {
    *lda = lda_;
    return A64_;
  }
  const float2* dense32(int64_t* lda) const override {
    *lda = lda32_;
    return A32_;
  }

 private:
  const double2* A64_;
  int64_t lda_;
  const float2* A32_;
  int64_t lda32_;
};

// Monostatic co-polarised (dirs NULL) or bistatic total RCS of nrhs current
// vectors j (nrhs x 2ne, canonical order, [alpha^M; alpha^J]) into rcs_host
// (nrhs x max(ndir, 1)); synchronises s.
void rcs_compute(const cbfm_mesh_s* m, const cbfm_medium* med, const double2* j, const double* inc, int64_t nrhs,
                 const double* dirs, int64_t ndir, double* rcs_host, hipStream_t s);


// v_r = (C^JM)^H v for nrhs tested incident fields v (cell order, nrhs x 2ne)
void project_rhs(const cbfm_mesh_s* m, cbfm_cbf_s* c, const double2* vint, int64_t nrhs, double2* b, hipStream_t s);
// j = C^MJ j_CBF (cell order, nrhs x 2ne)
void expand_cbf(const cbfm_mesh_s* m, cbfm_cbf_s* c, const double2* jc, int64_t nrhs, double2* jint, hipStream_t s);

// out[c][i] = in[c][perm[i]] (forward) or out[c][perm[i]] = in[c][i], both
// halves of 2ne-long vectors (the library's cell order <-> canonical order)
void permute_halves(const double2* in, double2* out, const int32_t* perm, int64_t ne, int64_t nv, int forward,
                    hipStream_t s);

}  // namespace cbfm
