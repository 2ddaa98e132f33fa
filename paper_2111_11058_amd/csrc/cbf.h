// CBF handle and the Calderon preconditioner (see cbf.hip).
#pragma once

#include <mutex>

#include "internal.h"

struct cbfm_cbf_s {
  const cbfm_mesh_s* mesh = nullptr;
  std::vector<int32_t> L;      // kept CBFs per cell (per current)
  std::vector<int64_t> off;    // prefix sums of L (nblocks + 1)
  std::vector<int64_t> coff;   // element offsets of cell blocks in CM / CJ (nblocks + 1)
  int64_t NL = 0;              // sum of L
  cbfm::DevBuf CM, CJ;         // per cell N_b x L_b row-major double2, cell after cell
  std::vector<double> sigma;   // kept singular values, cell after cell
  cbfm::DevBuf d_L, d_off, d_coff, d_cell_off, d_edge_block;
  // no triangle carries RWGs of two cells (disjoint bodies, one or more per
  // cell): the RWG Gram couples no two cells and B is block-diagonal by cell
  bool blockdiag = false;
  // built on a mesh of translated copies of cell 0: every cell holds cell
  // 0's CBFs (they span the same spaces), so a block of Z_r depends only on
  // the offset of its two cells
  bool shared = false;
  // B^{-1} for B = (C^M)^H G C^J (row-major), formed on first use
  std::mutex mu;
  bool factored = false;
  cbfm::DevBuf Binv;
  // after a CBF build, B^{-1} is formed on a side stream that overlaps the
  // caller's next work (the projection): `done` marks its end and dinfo
  // (ninfo entries, one per inverted block) its pivot checks, read at the
  // first use
  bool pending = false;
  hipEvent_t start = nullptr, done = nullptr;
  cbfm::DevBuf dinfo;
  int ninfo = 0;
  // the inexact CMP's operator G^CBF D^CBF (2NL x 2NL) and D^CBF, formed on
  // its first use (under mu)
  bool inner_ready = false;
  cbfm::DevBuf Gd, dinv;
  cbfm_cbf_s() = default;
  cbfm_cbf_s(const cbfm_cbf_s&) = delete;
  cbfm_cbf_s& operator=(const cbfm_cbf_s&) = delete;
  ~cbfm_cbf_s();  // waits for both events
};

namespace cbfm {

// Whether CBF builds on the calling thread queue the CMP inverse on a side
// stream (the default) or leave it to the first use (serving workers, whose
// requests already overlap one another).
void async_cmp_on_this_thread(bool on);
// x = GMRES solution of G^CBF x = y with the diagonal preconditioner
// D^CBF (right preconditioning, x0 = 0) to the relative residual tol
// (the paper's inexact inner CMP); y and x must not alias
void cmp_inner_apply(cbfm_cbf_s* c, int64_t nrhs, const double2* y, double2* x, double tol, hipStream_t s);
// x <- (G^CBF)^{-1} x in place, nrhs vectors of length 2 NL
void cmp_apply_dev(cbfm_cbf_s* c, int64_t nrhs, double2* x, hipStream_t s);
// B^{-1} (NL x NL, row-major), formed on first use
const double2* cmp_inverse(cbfm_cbf_s* c, hipStream_t s);
// Z_r of cbfm_project with an explicit scratch budget for the row panels
// CBFs of every cell from whole-body current coefficient sets (IPCBF): X
// holds S vectors of length 2 ne in the library's cell order, each
// [alpha^M; alpha^J]; cell m keeps its rows (Sec. III-A) and they are
// orthogonalised as in cbfm_build_cbf (Sec. III-B).  Synchronises s.
cbfm_cbf_s* cbf_from_currents(const cbfm_mesh_s* m, const double2* X, int S, double delta_svd, int max_L,
                              hipStream_t s);
// (returns the number of row panels)
int project_dev(const cbfm_mesh_s* m, const Media& md, cbfm_cbf_s* c, int precision, double2* Zr, int64_t ldz,
                hipStream_t s, size_t budget);

}  // namespace cbfm
