// The whole discretised PMCHWT system on one device, for the full-system
// uses of the method: the MoM baseline of the numerical section, the IPCBF
// generation, and the reduced operator applied without forming Z_r.
//
// Stored operator (the MoM arrangement with the diagonal preconditioner,
// Sec. IV, with the Buffa-Christiansen-tested T blocks read as the
// RWG-tested ones this fill computes):
//   A = Z_t D^{-1},  Z_t = [[-TE, K], [K, TH]] on j_t = [alpha^J; alpha^M],
//   D = diag(Z_t)
// with K = K1 + K2, TE = eta1 T1 + eta2 T2, TH = T1/eta1 + T2/eta2.  Z_t is
// the matrix Z of Sec. II-B with its two column blocks swapped (Z_t = Z P),
// so the plain product is Z u = A (D P^T u).  Rows are [E-tests; H-tests],
// columns [alpha^J; alpha^M], RWGs in the library's cell order.  The fill
// runs in row panels of whole cells (the triangle-local blocks of a panel's
// test triangles against every source triangle), assembled straight into
// A; then D is read off the diagonal and the columns are scaled.
//
//  * MoM baseline (cbfm_mom_solve): GMRES on A u = v, j_t = D^{-1} u.
//  * IPCBF (cbfm_build_ipcbf, Sec. III-A, the IPCBF equation solved by GMRES
//    with a loose allowance delta_r): the s generating waves solved on the
//    whole body; each cell keeps the rows of its RWGs, then the dual
//    orthogonalisation of Sec. III-B.
//  * Matrix-free reduced operator (cbfm_solve_matfree; Sec. III-C, the
//    remark after the current reconstruction): every GMRES product applies
//    (C^JM)^H Z C^MJ (G^CBF)^{-1} as five stages -- the CMP inverse, C^MJ per
//    cell, D P^T, the stored A, (C^JM)^H per cell -- and Z_r is never formed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "cbf.h"
#include "gemm.h"
#include "solve.h"

struct cbfm_mom_s {
  const cbfm_mesh_s* mesh = nullptr;
  cbfm_medium med{};
  int precision = CBFM_FP64;  // CBFM_FP64: A double; CBFM_FP32: A float (regular pairs filled in float)
  int64_t ne = 0, n = 0;
  cbfm::DevBuf A;  // n x n row-major (lda n)
  cbfm::DevBuf d;  // n double2: diag(Z_t)
};

namespace cbfm {

namespace {

template <typename R>
struct cz {
  R re, im;
};

// Rows r0 .. r0 + nrow - 1 of the E and H tests of A (before the column
// scaling) from a panel's triangle-local blocks (ops [K, TE, TH]): test RWG
// rowEdges[r], trial RWG colEdges[c] (every RWG, cell order).
template <typename R, typename RO>
__global__ void assemble_mom_kernel(const cz<R>* __restrict__ local, int64_t op_stride, int64_t ldl,
                                    const int32_t* __restrict__ rowEdges, int64_t r0, const int32_t* __restrict__ colEdges,
                                    int64_t ne, const int32_t* __restrict__ tplus, const int32_t* __restrict__ tminus,
                                    const int32_t* __restrict__ aplus, const int32_t* __restrict__ aminus,
                                    const int32_t* __restrict__ rowPos, cz<RO>* __restrict__ A) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= ne) return;
  const int32_t em = rowEdges[r], en = colEdges[c];
  const int64_t ri[2] = {3 * (int64_t)rowPos[tplus[em]] + aplus[em], 3 * (int64_t)rowPos[tminus[em]] + aminus[em]};
  const int64_t ci[2] = {3 * (int64_t)tplus[en] + aplus[en], 3 * (int64_t)tminus[en] + aminus[en]};
  RO v[3][2];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    RO re = 0, im = 0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const cz<R> e = local[o * op_stride + ri[x] * ldl + ci[y]];
        re += (RO)e.re;
        im += (RO)e.im;
      }
    v[o][0] = re;
    v[o][1] = im;
  }
  const int64_t n = 2 * ne, row = r0 + r;
  A[row * n + c] = cz<RO>{-v[1][0], -v[1][1]};       // E-test, alpha^J: -TE
  A[row * n + ne + c] = cz<RO>{v[0][0], v[0][1]};    // E-test, alpha^M: K
  A[(ne + row) * n + c] = cz<RO>{v[0][0], v[0][1]};  // H-test, alpha^J: K
  A[(ne + row) * n + ne + c] = cz<RO>{v[2][0], v[2][1]};  // H-test, alpha^M: TH
}

// d[i] = A[i][i]
template <typename RO>
__global__ void diag_kernel(const cz<RO>* __restrict__ A, int64_t n, double2* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cz<RO> a = A[i * n + i];
  d[i] = make_double2((double)a.re, (double)a.im);
}

// A[r][c] /= d[c] (in double); rows strided over the grid's y extent
template <typename RO>
__global__ void scale_columns_kernel(cz<RO>* __restrict__ A, int64_t n, const double2* __restrict__ d) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double2 q = d[c];
  const double den = q.x * q.x + q.y * q.y;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y) {
    const cz<RO> a = A[r * n + c];
    const double ar = (double)a.re, ai = (double)a.im;
    A[r * n + c] = cz<RO>{(RO)((ar * q.x + ai * q.y) / den), (RO)((ai * q.x - ar * q.y) / den)};
  }
}

// out[c][i] = u[c][k] / d[k], k = (i + ne) mod 2ne: j_t = D^{-1} u in the
// order [alpha^J; alpha^M] turned into [alpha^M; alpha^J]
__global__ void unscale_swap_kernel(const double2* __restrict__ u, const double2* __restrict__ d, double2* __restrict__ out,
                                    int64_t ne, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (i >= 2 * ne || c >= nv) return;
  const int64_t k = i < ne ? i + ne : i - ne;
  const double2 a = u[c * 2 * ne + k], q = d[k];
  const double den = q.x * q.x + q.y * q.y;
  out[c * 2 * ne + i] = make_double2((a.x * q.x + a.y * q.y) / den, (a.y * q.x - a.x * q.y) / den);
}

// out[c][k] = d[k] t[c][i], k = (i + ne) mod 2ne: D P^T t for t in the
// order [alpha^M; alpha^J] (the input of A for the plain product Z t)
__global__ void swap_scale_kernel(const double2* __restrict__ t, const double2* __restrict__ d, double2* __restrict__ out,
                                  int64_t ne, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (i >= 2 * ne || c >= nv) return;
  const int64_t k = i < ne ? i + ne : i - ne;
  const double2 a = t[c * 2 * ne + i], q = d[k];
  out[c * 2 * ne + k] = make_double2(a.x * q.x - a.y * q.y, a.x * q.y + a.y * q.x);
}

dim3 grid2(int64_t n, int64_t m) { return dim3((unsigned)((n + 255) / 256), (unsigned)m); }

// Fill and assemble A (then D and the scaling) in row panels of cells.
void build_operator(cbfm_mom_s* o, hipStream_t s, size_t budget) {
  const cbfm_mesh_s* m = o->mesh;
  const MeshHost& h = m->h;
  const Media md = make_media(&o->med);
  const int nb = h.nblocks;
  const int64_t ne = h.ne, nt = h.nt, n = 2 * ne;
  const int fillp = o->precision == CBFM_FP64 ? CBFM_FP64 : CBFM_FP32;
  const size_t esz = fillp == CBFM_FP64 ? 16 : 8;
  // panels of consecutive cells whose triangle-local blocks fit the budget
  std::vector<std::pair<int, int>> panels;
  {
    std::vector<int32_t> mark(nt, -1);
    int a0 = 0;
    while (a0 < nb) {
      int a1 = a0;
      int64_t nrt = 0;
      while (a1 < nb) {
        int64_t add = 0;
        for (int64_t i = h.cell_off[a1]; i < h.cell_off[a1 + 1]; ++i) {
          const int e = h.perm[i];
          for (int t : {h.tplus[e], h.tminus[e]})
            if (mark[t] != a0) {
              mark[t] = a0;
              ++add;
            }
        }
        if (a1 > a0 && (size_t)27 * (nrt + add) * nt * esz > budget) break;
        nrt += add;
        ++a1;
      }
      panels.push_back({a0, a1});
      a0 = a1;
    }
  }
  std::vector<int32_t> iota(nt);
  for (int64_t t = 0; t < nt; ++t) iota[t] = (int32_t)t;
  Scratch dcol((size_t)nt * sizeof(int32_t), s);
  CBFM_HIP(hipMemcpyAsync(dcol.p, iota.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, s));
  for (auto [p0, p1] : panels) {
    const int64_t r0 = h.cell_off[p0], nrow = h.cell_off[p1] - r0;
    std::vector<int32_t> pos(nt, -1), rows;
    for (int64_t i = r0; i < r0 + nrow; ++i) {
      pos[h.tplus[h.perm[i]]] = 0;
      pos[h.tminus[h.perm[i]]] = 0;
    }
    for (int64_t t = 0; t < nt; ++t)
      if (pos[t] == 0) {
        pos[t] = (int32_t)rows.size();
        rows.push_back((int32_t)t);
      }
    std::vector<NearPair> nl;
    for (const NearPair& q : h.near)
      if (pos[q.p] >= 0) nl.push_back({q.p, q.q, pos[q.p], q.q, q.coplanar, 0});
    const int64_t nrt = rows.size();
    const size_t ib = 4 * (rows.size() + pos.size()) + sizeof(NearPair) * nl.size();
    std::vector<char> host(ib);
    Scratch idx(ib, s);
    size_t off = 0;
    auto put = [&](const void* src, size_t bytes) {
      if (bytes) std::memcpy(host.data() + off, src, bytes);
      void* dst = idx.as<char>() + off;
      off += bytes;
      return dst;
    };
    auto* d_rows = (int32_t*)put(rows.data(), 4 * rows.size());
    auto* d_pos = (int32_t*)put(pos.data(), 4 * pos.size());
    auto* d_nl = (NearPair*)put(nl.data(), sizeof(NearPair) * nl.size());
    CBFM_HIP(hipMemcpyAsync(idx.p, host.data(), ib, hipMemcpyHostToDevice, s));
    Scratch local((size_t)27 * nrt * nt * esz, s);
    fill_local(m, md, fillp, CBFM_LAYOUT_OPS3, d_rows, nrt, dcol.as<int32_t>(), nt, d_nl, (int64_t)nl.size(), local.p, s);
    const int64_t ldl = 3 * nt, op_stride = 3 * nrt * ldl;
    CBFM_REQUIRE(nrow <= 65535, CBFM_E_ARG, "too many rows in one panel of cells");
    const dim3 grid((unsigned)((ne + 255) / 256), (unsigned)nrow);
    const int32_t *tp = m->tplus.as<int32_t>(), *tm = m->tminus.as<int32_t>();
    const int32_t *ap = m->aplus.as<int32_t>(), *am = m->aminus.as<int32_t>();
    TimedLaunch tl(T_ASSEMBLE, s);
    if (fillp == CBFM_FP64)
      hipLaunchKernelGGL((assemble_mom_kernel<double, double>), grid, dim3(256), 0, s, local.as<cz<double>>(), op_stride,
                         ldl, m->perm.as<int32_t>() + r0, r0, m->perm.as<int32_t>(), ne, tp, tm, ap, am, d_pos,
                         o->A.as<cz<double>>());
    else
      hipLaunchKernelGGL((assemble_mom_kernel<float, float>), grid, dim3(256), 0, s, local.as<cz<float>>(), op_stride,
                         ldl, m->perm.as<int32_t>() + r0, r0, m->perm.as<int32_t>(), ne, tp, tm, ap, am, d_pos,
                         o->A.as<cz<float>>());
    CBFM_HIP(hipGetLastError());
    CBFM_HIP(hipStreamSynchronize(s));  // host index staging of this panel
  }
  const dim3 g1((unsigned)((n + 255) / 256));
  CBFM_REQUIRE(n <= 0x7fffffffLL, CBFM_E_ARG, "system too large");
  if (fillp == CBFM_FP64) {
    hipLaunchKernelGGL(diag_kernel<double>, g1, dim3(256), 0, s, o->A.as<cz<double>>(), n, o->d.as<double2>());
    hipLaunchKernelGGL(scale_columns_kernel<double>, grid2(n, std::min<int64_t>(n, 4096)), dim3(256), 0, s,
                       o->A.as<cz<double>>(), n, o->d.as<double2>());
  } else {
    hipLaunchKernelGGL(diag_kernel<float>, g1, dim3(256), 0, s, o->A.as<cz<float>>(), n, o->d.as<double2>());
    hipLaunchKernelGGL(scale_columns_kernel<float>, grid2(n, std::min<int64_t>(n, 4096)), dim3(256), 0, s,
                       o->A.as<cz<float>>(), n, o->d.as<double2>());
  }
  CBFM_HIP(hipGetLastError());
  CBFM_HIP(hipStreamSynchronize(s));
}

// GMRES on A u = v for nrhs incidences or generating waves (canonical
// incidence rows, tested in the cell order), then j = [alpha^M; alpha^J]
// (cell order) = P D^{-1} u.  Returns the GMRES result.
GmresResult full_solve(const cbfm_mom_s* o, const double* inc_host, int64_t nrhs, const GmresSpec& sp, double2* jz,
                       hipStream_t s) {
  const cbfm_mesh_s* m = o->mesh;
  const Media md = make_media(&o->med);
  const int64_t ne = o->ne, n = o->n;
  Scratch dinc(nrhs * 6 * sizeof(double), s);
  CBFM_HIP(hipMemcpyAsync(dinc.p, inc_host, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, s));
  Scratch v(nrhs * n * sizeof(double2), s), vint(nrhs * n * sizeof(double2), s), u(nrhs * n * sizeof(double2), s);
  rhs_launch(m, md, o->med.eta0, dinc.as<double>(), nrhs, v.p, s);
  permute_halves(v.as<double2>(), vint.as<double2>(), m->perm.as<int32_t>(), ne, nrhs, 1, s);
  DenseOp op(o->precision == CBFM_FP64 ? o->A.as<double2>() : nullptr, n,
             o->precision == CBFM_FP64 ? nullptr : o->A.as<float2>(), n);
  GmresResult r = gmres_run(op, n, nrhs, vint.as<double2>(), u.as<double2>(), sp, s);
  hipLaunchKernelGGL(unscale_swap_kernel, grid2(n, nrhs), dim3(256), 0, s, u.as<double2>(), o->d.as<double2>(), jz, ne,
                     nrhs);
  CBFM_HIP(hipGetLastError());
  CBFM_HIP(hipStreamSynchronize(s));
  return r;
}

// The reduced operator (C^JM)^H Z C^MJ [(G^CBF)^{-1}] applied in stages
// from the stored A (matrix-free: Z_r is never formed).
class MatFreeReduced : public KrylovOp {
 public:
  MatFreeReduced(const cbfm_mom_s* o, cbfm_cbf_s* c, bool cmp, int64_t nrhs, hipStream_t s)
      : o_(o), c_(c), cmp_(cmp), nrhs_(nrhs), NL_(c->NL), t0_(cmp ? nrhs * 2 * c->NL * sizeof(double2) : 0, s),
        t1_(nrhs * o->n * sizeof(double2), s), t2_(nrhs * o->n * sizeof(double2), s),
        t3_(nrhs * o->n * sizeof(double2), s) {
    if (cmp_) Bi_ = cmp_inverse(c, s);
  }
  void prepare(const double2* V, int64_t vstride, double2* w, int64_t mres, int64_t nrhs, hipStream_t s) override {
    std::vector<std::vector<GemmDesc>> g;
    for (int64_t j = 0; j < mres; ++j) g.push_back(first_stage(V + j * vstride));
    plan_first_.reset(new GemmPlan(g, s, false));
    build_tail(w, s);
    (void)nrhs;
  }
  void launch(int64_t j, hipStream_t q) const override {
    plan_first_->launch((size_t)j, q);
    run_tail(q);
  }
  void apply(const double2* x, double2* r, int64_t nrhs, hipStream_t s) const override {
    (void)nrhs;
    std::vector<GemmDesc> f = first_stage(x);
    zgemm_batched(f, s);
    std::vector<GemmDesc> expand = expand_descs(), mat = matvec_descs(), back = back_descs(r);
    if (cmp_) zgemm_batched(expand, s);
    swap_scale(s);
    if (o_->precision == CBFM_FP64) {
      zgemm_batched(mat, s);
    } else {
      std::vector<GemmDescX> mx = matvec_descs32();
      xgemm_batched(mx, XG_FP32, s);
    }
    zgemm_batched(back, s);
  }

 private:
  const cbfm_mom_s* o_;
  cbfm_cbf_s* c_;
  bool cmp_;
  int64_t nrhs_, NL_;
  const double2* Bi_ = nullptr;
  Scratch t0_, t1_, t2_, t3_;
  std::unique_ptr<GemmPlan> plan_first_, plan_expand_, plan_mat_, plan_back_;
  std::unique_ptr<XGemmPlan> plan_mat32_;

  const MeshHost& h() const { return o_->mesh->h; }
  // first stage from the input q: with the CMP, t0 = (G^CBF)^{-1} q
  // (blkdiag(-(B^{-1})^H, B^{-1}), as the CMP apply); else straight into
  // t1 = C^MJ q
  std::vector<GemmDesc> first_stage(const double2* q) const {
    const int64_t nr = 2 * NL_;
    if (cmp_)
      return {gemm(q, nr, OP_N, Bi_, NL_, OP_R, t0_.as<double2>(), nr, nrhs_, NL_, NL_, -1.0),
              gemm(q + NL_, nr, OP_N, Bi_, NL_, OP_T, t0_.as<double2>() + NL_, nr, nrhs_, NL_, NL_)};
    return expand_from(q);
  }
  // t1 = C^MJ src (per cell; rows = vectors)
  std::vector<GemmDesc> expand_from(const double2* src) const {
    const int64_t ne = o_->ne, nr = 2 * NL_;
    std::vector<GemmDesc> ds;
    for (int a = 0; a < h().nblocks; ++a) {
      const int64_t Na = h().cell_off[a + 1] - h().cell_off[a], r0 = h().cell_off[a];
      ds.push_back(gemm(src + c_->off[a], nr, OP_N, c_->CM.as<double2>() + c_->coff[a], c_->L[a], OP_T,
                        t1_.as<double2>() + r0, 2 * ne, nrhs_, Na, c_->L[a]));
      ds.push_back(gemm(src + NL_ + c_->off[a], nr, OP_N, c_->CJ.as<double2>() + c_->coff[a], c_->L[a], OP_T,
                        t1_.as<double2>() + ne + r0, 2 * ne, nrhs_, Na, c_->L[a]));
    }
    return ds;
  }
  std::vector<GemmDesc> expand_descs() const { return expand_from(t0_.as<double2>()); }
  // t3 = A t2 (rows = vectors)
  std::vector<GemmDesc> matvec_descs() const {
    const int64_t n = o_->n;
    GemmDesc d = gemm(o_->A.as<double2>(), n, OP_N, t2_.as<double2>(), n, OP_T, t3_.as<double2>(), n, n, nrhs_, n);
    d.transC = 1;
    return {d};
  }
  std::vector<GemmDescX> matvec_descs32() const {
    const int64_t n = o_->n;
    GemmDescX d = gemmx(o_->A.as<float2>(), 0, n, OP_N, t2_.as<double2>(), 1, n, OP_T, t3_.as<double2>(), 1, n, n,
                        nrhs_, n);
    d.transC = 1;
    return {d};
  }
  // w = (C^JM)^H t3 (per cell)
  std::vector<GemmDesc> back_descs(double2* w) const {
    const int64_t ne = o_->ne, nr = 2 * NL_;
    std::vector<GemmDesc> ds;
    for (int a = 0; a < h().nblocks; ++a) {
      const int64_t Na = h().cell_off[a + 1] - h().cell_off[a], r0 = h().cell_off[a];
      ds.push_back(gemm(t3_.as<double2>() + r0, 2 * ne, OP_N, c_->CJ.as<double2>() + c_->coff[a], c_->L[a], OP_R,
                        w + c_->off[a], nr, nrhs_, c_->L[a], Na));
      ds.push_back(gemm(t3_.as<double2>() + ne + r0, 2 * ne, OP_N, c_->CM.as<double2>() + c_->coff[a], c_->L[a], OP_R,
                        w + NL_ + c_->off[a], nr, nrhs_, c_->L[a], Na));
    }
    return ds;
  }
  void swap_scale(hipStream_t q) const {
    hipLaunchKernelGGL(swap_scale_kernel, grid2(o_->n, nrhs_), dim3(256), 0, q, t1_.as<double2>(), o_->d.as<double2>(),
                       t2_.as<double2>(), o_->ne, nrhs_);
    CBFM_HIP(hipGetLastError());
  }
  void build_tail(double2* w, hipStream_t s) {
    if (cmp_) plan_expand_.reset(new GemmPlan({expand_descs()}, s, false));
    if (o_->precision == CBFM_FP64)
      plan_mat_.reset(new GemmPlan({matvec_descs()}, s, false));
    else
      plan_mat32_.reset(new XGemmPlan({matvec_descs32()}, XG_FP32, s));
    plan_back_.reset(new GemmPlan({back_descs(w)}, s, false));
  }
  void run_tail(hipStream_t q) const {
    if (plan_expand_) plan_expand_->launch(0, q);
    swap_scale(q);
    if (plan_mat_)
      plan_mat_->launch(0, q);
    else
      plan_mat32_->launch(0, q);
    plan_back_->launch(0, q);
  }
};

}  // namespace

}  // namespace cbfm

using namespace cbfm;

extern "C" {

cbfm_status cbfm_mom_build(cbfm_mesh m, const cbfm_medium* med, int32_t precision, int64_t panel_bytes, void* stream,
                           cbfm_mom* out) {
  return guarded([&] {
    CBFM_REQUIRE(m && med && out, CBFM_E_ARG, "null argument");
    *out = nullptr;
    CBFM_REQUIRE(precision == CBFM_FP64 || precision == CBFM_FP32, CBFM_E_ARG, "precision must be FP64 or FP32");
    CBFM_REQUIRE(panel_bytes >= 0, CBFM_E_ARG, "negative panel budget");
    (void)make_media(med);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto o = std::make_unique<cbfm_mom_s>();
    o->mesh = m;
    o->med = *med;
    o->precision = precision;
    o->ne = m->h.ne;
    o->n = 2 * m->h.ne;
    const size_t esz = precision == CBFM_FP64 ? sizeof(double2) : sizeof(float2);
    o->A.alloc((size_t)o->n * o->n * esz);
    o->d.alloc((size_t)o->n * sizeof(double2));
    size_t budget = (size_t)panel_bytes;
    if (budget == 0) {
      size_t fr = 0, tot = 0;
      CBFM_HIP(hipMemGetInfo(&fr, &tot));
      fr += scratch_cached_bytes();
      budget = std::min<size_t>(fr / 4, (size_t)32 << 30);
    }
    build_operator(o.get(), s, budget);
    *out = o.release();
  });
}

cbfm_status cbfm_mom_info(cbfm_mom o, int64_t* n, int32_t* precision) {
  return guarded([&] {
    CBFM_REQUIRE(o != nullptr, CBFM_E_ARG, "null operator");
    if (n) *n = o->n;
    if (precision) *precision = o->precision;
  });
}

cbfm_status cbfm_mom_export(cbfm_mom o, int64_t row0, int64_t nrow, void* A_dev, int64_t ld, void* d_dev,
                            void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(o != nullptr, CBFM_E_ARG, "null operator");
    CBFM_REQUIRE(row0 >= 0 && nrow >= 0 && row0 + nrow <= o->n, CBFM_E_ARG, "rows outside [0, n)");
    CBFM_REQUIRE(A_dev == nullptr || ld >= o->n, CBFM_E_ARG, "ld < n");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t esz = o->precision == CBFM_FP64 ? sizeof(double2) : sizeof(float2);
    if (A_dev && nrow > 0)
      CBFM_HIP(hipMemcpy2DAsync(A_dev, (size_t)ld * esz, o->A.as<char>() + (size_t)row0 * o->n * esz, (size_t)o->n * esz,
                                (size_t)o->n * esz, (size_t)nrow, hipMemcpyDeviceToDevice, s));
    if (d_dev) CBFM_HIP(hipMemcpyAsync(d_dev, o->d.p, (size_t)o->n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  });
}

void cbfm_mom_free(cbfm_mom o) { delete o; }

cbfm_status cbfm_mom_solve(cbfm_mom o, const double* inc, int64_t nrhs, const cbfm_solver_params* prm, void* j_dev,
                           int32_t* iters, double* relres, const double* dirs, int64_t ndir, double* rcs, void* stream) {
  bool noconv = false;
  const cbfm_status st = guarded([&] {
    CBFM_REQUIRE(o && inc && prm, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, CBFM_E_ARG, "nrhs out of range");
    CBFM_REQUIRE(prm->tol > 0 && prm->max_iter >= 1 && prm->restart >= 1, CBFM_E_ARG, "bad solver parameters");
    CBFM_REQUIRE(prm->sstep == 0, CBFM_E_ARG, "s-step cycles are a cbfm_solve form");
    CBFM_REQUIRE(prm->block == 0 || (prm->block >= 1 && prm->block <= 32 && prm->inner_fp32 == 0 &&
                                     prm->basis_fp32 == 0 && prm->use_graph == 0 && o->precision == CBFM_FP64),
                 CBFM_E_ARG, "block is 0 to 32, with the FP64 operator, double cycles and no graphs");
    CBFM_REQUIRE(dirs == nullptr || ndir >= 1, CBFM_E_ARG, "ndir must be >= 1 with dirs");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const cbfm_mesh_s* m = o->mesh;
    GmresSpec sp;
    sp.tol = prm->tol;
    sp.max_iter = prm->max_iter;
    sp.restart = prm->restart;
    sp.f32 = prm->inner_fp32 != 0;
    sp.inner_tol = prm->inner_tol;
    sp.graph = prm->use_graph != 0;
    sp.basis32 = prm->basis_fp32 != 0 && prm->inner_fp32 == 0;
    sp.block = prm->block;
    Scratch jz(nrhs * o->n * sizeof(double2), s), jout(nrhs * o->n * sizeof(double2), s);
    const GmresResult r = full_solve(o, inc, nrhs, sp, jz.as<double2>(), s);
    noconv = r.noconv;
    double2* jfinal = j_dev ? static_cast<double2*>(j_dev) : jout.as<double2>();
    permute_halves(jz.as<double2>(), jfinal, m->perm.as<int32_t>(), o->ne, nrhs, 0, s);
    if (rcs) rcs_compute(m, &o->med, jfinal, inc, nrhs, dirs, ndir, rcs, s);
    CBFM_HIP(hipStreamSynchronize(s));
    if (iters) std::memcpy(iters, r.its.data(), nrhs * sizeof(int32_t));
    if (relres) std::memcpy(relres, r.res.data(), nrhs * sizeof(double));
    if (noconv) set_error("GMRES did not reach the tolerance for every right-hand side");
  });
  return st != CBFM_OK ? st : (noconv ? CBFM_E_NOCONV : CBFM_OK);
}

cbfm_status cbfm_build_ipcbf(cbfm_mom o, const cbfm_ipcbf_params* prm, void* stream, cbfm_cbf* out, int32_t* iters,
                             double* relres) {
  return guarded([&] {
    CBFM_REQUIRE(o && prm && out, CBFM_E_ARG, "null argument");
    *out = nullptr;
    CBFM_REQUIRE(prm->gen_host && prm->n_gen >= 1 && prm->n_gen <= 4096, CBFM_E_ARG, "need 1 to 4096 generating waves");
    CBFM_REQUIRE(prm->delta_r > 0 && prm->delta_r < 1, CBFM_E_ARG, "delta_r outside (0, 1)");
    CBFM_REQUIRE(prm->delta_svd >= 0 && prm->delta_svd <= 1, CBFM_E_ARG, "delta_svd outside [0, 1]");
    CBFM_REQUIRE(prm->max_iter >= 1, CBFM_E_ARG, "max_iter must be positive");
    CBFM_REQUIRE(prm->block >= 0 && prm->block <= 32, CBFM_E_ARG, "block must be 0, 1 or a group size up to 32");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t S = prm->n_gen;
    GmresSpec sp;
    sp.tol = prm->delta_r;
    sp.max_iter = prm->max_iter;
    sp.restart = prm->restart > 0 ? prm->restart : prm->max_iter;
    sp.block = prm->block;
    Scratch jz(S * o->n * sizeof(double2), s);
    const GmresResult r = full_solve(o, prm->gen_host, S, sp, jz.as<double2>(), s);
    if (iters) std::memcpy(iters, r.its.data(), S * sizeof(int32_t));
    if (relres) std::memcpy(relres, r.res.data(), S * sizeof(double));
    CBFM_REQUIRE(!r.noconv, CBFM_E_NOCONV, "a generating wave did not reach delta_r within max_iter");
    *out = cbf_from_currents(o->mesh, jz.as<double2>(), (int)S, prm->delta_svd, prm->max_L, s);
  });
}

cbfm_status cbfm_solve_matfree(cbfm_mom o, cbfm_cbf c, const double* inc, int64_t nrhs, const cbfm_solver_params* prm,
                               void* j_dev, int32_t* iters, double* relres, const double* dirs, int64_t ndir,
                               double* rcs, void* stream) {
  bool noconv = false;
  const cbfm_status st = guarded([&] {
    CBFM_REQUIRE(o && c && inc && prm, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(c->mesh == o->mesh, CBFM_E_STATE, "CBF set belongs to another mesh");
    CBFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, CBFM_E_ARG, "nrhs out of range");
    CBFM_REQUIRE(prm->tol > 0 && prm->max_iter >= 1 && prm->restart >= 1, CBFM_E_ARG, "bad solver parameters");
    CBFM_REQUIRE(prm->use_cmp == 0 || prm->use_cmp == 1, CBFM_E_ARG, "use_cmp must be 0 or 1");
    CBFM_REQUIRE(prm->cmp_mode == CBFM_CMP_EXACT, CBFM_E_ARG, "the matrix-free operator takes the exact CMP");
    CBFM_REQUIRE(prm->inner_fp32 == 0 && prm->use_graph == 0 && prm->basis_fp32 == 0 && prm->sstep == 0 &&
                     prm->block == 0, CBFM_E_ARG,
                 "the matrix-free operator runs double Krylov cycles with a double basis and without graphs");
    CBFM_REQUIRE(dirs == nullptr || ndir >= 1, CBFM_E_ARG, "ndir must be >= 1 with dirs");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const cbfm_mesh_s* m = o->mesh;
    const Media md = make_media(&o->med);
    const int64_t ne = o->ne, NL = c->NL, n = 2 * NL;
    Scratch dinc(nrhs * 6 * sizeof(double), s);
    CBFM_HIP(hipMemcpyAsync(dinc.p, inc, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, s));
    Scratch v(nrhs * 2 * ne * sizeof(double2), s), vint(nrhs * 2 * ne * sizeof(double2), s), b(nrhs * n * sizeof(double2), s);
    rhs_launch(m, md, o->med.eta0, dinc.as<double>(), nrhs, v.p, s);
    permute_halves(v.as<double2>(), vint.as<double2>(), m->perm.as<int32_t>(), ne, nrhs, 1, s);
    project_rhs(m, c, vint.as<double2>(), nrhs, b.as<double2>(), s);
    MatFreeReduced op(o, c, prm->use_cmp != 0, nrhs, s);
    GmresSpec sp;
    sp.tol = prm->tol;
    sp.max_iter = prm->max_iter;
    sp.restart = prm->restart;
    Scratch x(nrhs * n * sizeof(double2), s);
    const GmresResult r = gmres_run(op, n, nrhs, b.as<double2>(), x.as<double2>(), sp, s);
    noconv = r.noconv;
    if (prm->use_cmp) cmp_apply_dev(c, nrhs, x.as<double2>(), s);
    Scratch jint(nrhs * 2 * ne * sizeof(double2), s), jout(nrhs * 2 * ne * sizeof(double2), s);
    expand_cbf(m, c, x.as<double2>(), nrhs, jint.as<double2>(), s);
    double2* jfinal = j_dev ? static_cast<double2*>(j_dev) : jout.as<double2>();
    permute_halves(jint.as<double2>(), jfinal, m->perm.as<int32_t>(), ne, nrhs, 0, s);
    if (rcs) rcs_compute(m, &o->med, jfinal, inc, nrhs, dirs, ndir, rcs, s);
    CBFM_HIP(hipStreamSynchronize(s));
    if (iters) std::memcpy(iters, r.its.data(), nrhs * sizeof(int32_t));
    if (relres) std::memcpy(relres, r.res.data(), nrhs * sizeof(double));
    if (noconv) set_error("GMRES did not reach the tolerance for every right-hand side");
  });
  return st != CBFM_OK ? st : (noconv ? CBFM_E_NOCONV : CBFM_OK);
}

}  // extern "C"
