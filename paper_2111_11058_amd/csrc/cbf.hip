// Characteristic basis functions with dual orthogonalisation (paper Sec.
// III-A, III-B) and the Calderon preconditioner G^CBF (Sec. III-C).
//
// build:  per cell m
//   Z_mm   = cell block of [[K, -TE], [TH, K]]            (fill kernels, FP64)
//   J_m    = Z_mm^{-1} V_m  for the generating waves      (batched LU)
//   G'_m   = (J^M)^H G_m J^J, G_m the rotated RWG Gram
//   G'_m   = U S V^H, keep sigma_i / sigma_1 >= delta_svd
//   C^M_m  = J^M U_L,  C^J_m = J^J V_L
// The SVD is taken of an r x r core, r = min(s, N_m): with the QR
// factorisations (J^M)^H = Q_M R_M and (J^J)^H = Q_J R_J (batched geqrf),
// G'_m = Q_M (R_M G_m R_J^H) Q_J^H, so with R_M G_m R_J^H = U_c S V_c^H the
// singular values are those of G'_m and, since J^M Q_M = R_M^H,
// C^M_m = R_M^H U_c,L and C^J_m = R_J^H V_c,L (matrix-core GEMMs).
// G_m is taken in closed form: for two RWGs a != b of one triangle with
// counter-clockwise local indices, int (n x f_a) . f_b = e_ab l_a l_b / 6
// times the RWG signs, e_ab = +1 if b follows a cyclically, -1 otherwise;
// it is zero on the diagonal and for RWGs sharing no triangle.
//
// G^CBF = blkdiag(A, B) with B = (C^M)^H G C^J and A = (C^J)^H G C^M =
// -B^H (G real antisymmetric), so one inverse of B serves both halves.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "cbf.h"
#include "gemm.h"

namespace cbfm {

// ------------------------------------------------------------- rocSOLVER handle
static std::mutex g_blas_mu;

rocblas_handle blas_handle(hipStream_t s) {
  static std::map<int, rocblas_handle> handles;
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  auto it = handles.find(dev);
  if (it == handles.end()) {
    rocblas_handle h;
    CBFM_REQUIRE(rocblas_create_handle(&h) == rocblas_status_success, CBFM_E_HIP, "rocblas_create_handle failed");
    it = handles.emplace(dev, h).first;
  }
  CBFM_REQUIRE(rocblas_set_stream(it->second, s) == rocblas_status_success, CBFM_E_HIP, "rocblas_set_stream failed");
  return it->second;
}

std::mutex& blas_mutex() { return g_blas_mu; }

#define CBFM_RS(call)                                                                                  \
  do {                                                                                                 \
    rocblas_status st_ = (call);                                                                       \
    CBFM_REQUIRE(st_ == rocblas_status_success, CBFM_E_HIP,                                            \
                 std::string(#call) + ": rocblas status " + std::to_string((int)st_));                 \
  } while (0)

// ------------------------------------------------------------- kernels
// Gram entry G[e, f] of two canonical edges (closed form above).
__device__ double gram_entry(int e, int f, const int32_t* tplus, const int32_t* tminus, const int32_t* aplus,
                             const int32_t* aminus, const int32_t* tri_edge, const int32_t* tri_sign,
                             const double* length) {
  if (e == f) return 0.0;
  double g = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int t = side ? tminus[e] : tplus[e];
    const int a = side ? aminus[e] : aplus[e];
    for (int db = 1; db <= 2; ++db) {
      const int b = (a + db) % 3;
      if (tri_edge[t * 3 + b] == f) {
        const double eps = db == 1 ? 1.0 : -1.0;
        g += eps * length[e] * length[f] / 6.0 * tri_sign[t * 3 + a] * tri_sign[t * 3 + b];
      }
    }
  }
  return g;
}

// Dense cell Gram G_m (N x N complex, row-major) for canonical edge list `ed`.
__global__ void cell_gram_kernel(const int32_t* __restrict__ ed, int N, const int32_t* tplus, const int32_t* tminus,
                                 const int32_t* aplus, const int32_t* aminus, const int32_t* tri_edge,
                                 const int32_t* tri_sign, const double* length, double2* __restrict__ G) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= N) return;
  G[(int64_t)r * N + c] =
      make_double2(gram_entry(ed[r], ed[c], tplus, tminus, aplus, aminus, tri_edge, tri_sign, length), 0.0);
}

// Pack the cell block of [[K, -TE], [TH, K]] (from 3 x N x N row-major) into
// a column-major n x n matrix with identity padding.
__global__ void pack_zmm_kernel(const double2* __restrict__ ops, int N, int n, double2* __restrict__ Z) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r >= n) return;
  double2 v = make_double2(r == c ? 1.0 : 0.0, 0.0);
  if (r < 2 * N && c < 2 * N) {
    const int br = r / N, bc = c / N, rr = r % N, cc = c % N;
    const int64_t NN = (int64_t)N * N;
    // [[K, -TE], [TH, K]] with ops = [K, TE, TH]
    const int op = (br == bc) ? 0 : (br == 0 ? 1 : 2);
    v = ops[op * NN + (int64_t)rr * N + cc];
    if (br == 0 && bc == 1) {
      v.x = -v.x;
      v.y = -v.y;
    }
  }
  Z[(int64_t)c * n + r] = v;
}

// Pack the generating right-hand sides of a cell: column c of the n x s
// column-major block is [v^E(edges); v^H(edges); 0].
__global__ void pack_v_kernel(const double2* __restrict__ v, int64_t ne, const int32_t* __restrict__ ed, int N,
                              int n, double2* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r >= n) return;
  double2 x = make_double2(0.0, 0.0);
  if (r < N)
    x = v[(int64_t)c * 2 * ne + ed[r]];
  else if (r < 2 * N)
    x = v[(int64_t)c * 2 * ne + ne + ed[r - N]];
  out[(int64_t)c * n + r] = x;
}

// From a cell's solved currents J = [J^M; J^J] (column-major n x S, the
// magnetic rows first), write (J^M)^H and (J^J)^H as column-major S x Nmax
// matrices (blockIdx.z picks which), zero beyond the cell's N columns.
__global__ void pack_jh_kernel(const double2* __restrict__ J, int n, int S, int N, int Nmax,
                               double2* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y, w = blockIdx.z;
  if (r >= S) return;
  double2 x = make_double2(0.0, 0.0);
  if (c < N) {
    x = J[(int64_t)r * n + w * N + c];
    x.y = -x.y;
  }
  out[(int64_t)w * S * Nmax + (int64_t)c * S + r] = x;
}

// Row-major r x Nmax copy of the triangular factor that geqrf left in the
// upper triangle of a column-major S x Nmax matrix (blockIdx.z: M or J).
__global__ void extract_r_kernel(const double2* __restrict__ qr, int S, int N, int Nmax, int rk,
                                 double2* __restrict__ R) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y, w = blockIdx.z;
  if (j >= Nmax) return;
  double2 x = make_double2(0.0, 0.0);
  if (i <= j && j < N) x = qr[(int64_t)w * S * Nmax + (int64_t)j * S + i];
  R[(int64_t)w * rk * Nmax + (int64_t)i * Nmax + j] = x;
}

// GC[m][col] = sum_n G[perm[m], n] C^J_full[n][col], rows in internal order.
__global__ void gram_times_cj_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
                                     const int32_t* __restrict__ edge_block, const int64_t* __restrict__ cell_off,
                                     const int64_t* __restrict__ off, const int32_t* __restrict__ L,
                                     const int64_t* __restrict__ coff, const double2* __restrict__ CJ, int64_t ne,
                                     int64_t NL, const int32_t* tplus, const int32_t* tminus, const int32_t* aplus,
                                     const int32_t* aminus, const int32_t* tri_edge, const int32_t* tri_sign,
                                     const double* length, double2* __restrict__ GC) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, m = blockIdx.y;
  if (col >= NL) return;
  const int e = perm[m];
  double2 acc = make_double2(0.0, 0.0);
  for (int side = 0; side < 2; ++side) {
    const int t = side ? tminus[e] : tplus[e];
    const int a = side ? aminus[e] : aplus[e];
    for (int db = 1; db <= 2; ++db) {
      const int b = (a + db) % 3;
      const int f = tri_edge[t * 3 + b];
      const double g = (db == 1 ? 1.0 : -1.0) * length[e] * length[f] / 6.0 * tri_sign[t * 3 + a] * tri_sign[t * 3 + b];
      const int cf = edge_block[f];
      if (col >= off[cf] && col < off[cf] + L[cf]) {
        const int64_t row = iperm[f] - cell_off[cf];
        const double2 c = CJ[coff[cf] + row * L[cf] + (col - off[cf])];
        acc.x += g * c.x;
        acc.y += g * c.y;
      }
    }
  }
  GC[m * NL + col] = acc;
}

// ------------------------------------------------------------- host helpers
static std::vector<int32_t> cell_edges(const MeshHost& h, int b) {
  return std::vector<int32_t>(h.perm.begin() + h.cell_off[b], h.perm.begin() + h.cell_off[b + 1]);
}

void cbf_finish(cbfm_cbf_s* c) {
  const MeshHost& h = c->mesh->h;
  c->off.assign(h.nblocks + 1, 0);
  c->coff.assign(h.nblocks + 1, 0);
  for (int b = 0; b < h.nblocks; ++b) {
    c->off[b + 1] = c->off[b] + c->L[b];
    c->coff[b + 1] = c->coff[b] + (h.cell_off[b + 1] - h.cell_off[b]) * (int64_t)c->L[b];
  }
  c->NL = c->off[h.nblocks];
  c->d_L.upload(c->L);
  c->d_off.upload(c->off);
  c->d_coff.upload(c->coff);
  c->d_cell_off.upload(h.cell_off);
  c->d_edge_block.upload(h.edge_block);
}

// B^{-1} for B = (C^M)^H G C^J.  rocSOLVER works column-major, so it sees
// M = B^T; LU + inversion of M leaves M^{-1} = (B^{-1})^T in column-major
// order, i.e. B^{-1} in the row-major layout used here.
static void cmp_factor(cbfm_cbf_s* c, hipStream_t s) {
  const cbfm_mesh_s* m = c->mesh;
  const MeshHost& h = m->h;
  const int64_t NL = c->NL, ne = h.ne;
  Scratch GC(ne * NL * sizeof(double2), s);
  dim3 grid((unsigned)((NL + 255) / 256), (unsigned)ne);
  hipLaunchKernelGGL(gram_times_cj_kernel, grid, dim3(256), 0, s, m->perm.as<int32_t>(), m->iperm.as<int32_t>(),
                     c->d_edge_block.as<int32_t>(), c->d_cell_off.as<int64_t>(), c->d_off.as<int64_t>(),
                     c->d_L.as<int32_t>(), c->d_coff.as<int64_t>(), c->CJ.as<double2>(), ne, NL,
                     m->tplus.as<int32_t>(), m->tminus.as<int32_t>(), m->aplus.as<int32_t>(), m->aminus.as<int32_t>(),
                     m->tri_edge.as<int32_t>(), m->tri_sign.as<int32_t>(), m->length.as<double>(), GC.as<double2>());
  CBFM_HIP(hipGetLastError());
  c->Binv.alloc(NL * NL * sizeof(double2));
  std::vector<GemmDesc> ds;
  for (int a = 0; a < h.nblocks; ++a) {
    const int64_t Na = h.cell_off[a + 1] - h.cell_off[a];
    ds.push_back(gemm(c->CM.as<double2>() + c->coff[a], c->L[a], OP_C, GC.as<double2>() + h.cell_off[a] * NL, NL,
                      OP_N, c->Binv.as<double2>() + c->off[a] * NL, NL, c->L[a], NL, Na));
  }
  zgemm_batched(ds, s);
  Scratch ipiv(NL * sizeof(rocblas_int), s);
  Scratch info(2 * sizeof(rocblas_int), s);
  {
    std::lock_guard<std::mutex> lk(blas_mutex());
    rocblas_handle bh = blas_handle(s);
    CBFM_RS(rocsolver_zgetrf(bh, (rocblas_int)NL, (rocblas_int)NL, (rocblas_double_complex*)c->Binv.p,
                             (rocblas_int)NL, ipiv.as<rocblas_int>(), info.as<rocblas_int>()));
    CBFM_RS(rocsolver_zgetri(bh, (rocblas_int)NL, (rocblas_double_complex*)c->Binv.p, (rocblas_int)NL,
                             ipiv.as<rocblas_int>(), info.as<rocblas_int>() + 1));
  }
  rocblas_int hinfo[2] = {0, 0};
  CBFM_HIP(hipMemcpyAsync(hinfo, info.p, sizeof(hinfo), hipMemcpyDeviceToHost, s));
  CBFM_HIP(hipStreamSynchronize(s));
  CBFM_REQUIRE(hinfo[0] == 0 && hinfo[1] == 0, CBFM_E_RANK,
               "G^CBF is singular (zero pivot " + std::to_string(hinfo[0]) + ")");
  c->factored = true;
}

const double2* cmp_inverse(cbfm_cbf_s* c, hipStream_t s) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->factored) cmp_factor(c, s);
  return c->Binv.as<double2>();
}

// x <- (G^CBF)^{-1} x with (G^CBF)^{-1} = blkdiag(-(B^{-1})^H, B^{-1}); for
// vectors stored as rows: x1 <- -x1 conj(B^{-1}),  x2 <- x2 (B^{-1})^T.
void cmp_apply_dev(cbfm_cbf_s* c, int64_t nrhs, double2* x, hipStream_t s) {
  const double2* Bi = cmp_inverse(c, s);
  const int64_t NL = c->NL, n = 2 * NL;
  if (nrhs == 0 || NL == 0) return;
  Scratch y(nrhs * n * sizeof(double2), s);
  CBFM_HIP(hipMemcpyAsync(y.p, x, nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  std::vector<GemmDesc> ds{gemm(y.as<double2>(), n, OP_N, Bi, NL, OP_R, x, n, nrhs, NL, NL, -1.0),
                           gemm(y.as<double2>() + NL, n, OP_N, Bi, NL, OP_T, x + NL, n, nrhs, NL, NL)};
  zgemm_batched(ds, s);
}

// Per-cell support triangles and the near pairs inside it.
struct CellSupport {
  std::vector<int32_t> tris, pos, edges;
  std::vector<NearPair> near;
};

static CellSupport support(const MeshHost& h, const std::vector<int32_t>& edges) {
  CellSupport cs;
  cs.edges = edges;
  cs.pos.assign(h.nt, -1);
  for (int32_t e : edges) {
    cs.pos[h.tplus[e]] = 0;
    cs.pos[h.tminus[e]] = 0;
  }
  for (int64_t t = 0; t < h.nt; ++t)
    if (cs.pos[t] == 0) {
      cs.pos[t] = (int32_t)cs.tris.size();
      cs.tris.push_back((int32_t)t);
    }
  for (const NearPair& q : h.near)
    if (cs.pos[q.p] >= 0 && cs.pos[q.q] >= 0) cs.near.push_back({q.p, q.q, cs.pos[q.p], cs.pos[q.q], q.coplanar, 0});
  return cs;
}

}  // namespace cbfm

using namespace cbfm;

extern "C" {

cbfm_status cbfm_build_cbf(cbfm_mesh m, const cbfm_medium* med, const cbfm_cbf_params* prm, void* stream,
                           cbfm_cbf* out) {
  return guarded([&] {
    CBFM_REQUIRE(m && prm && out, CBFM_E_ARG, "null argument");
    *out = nullptr;
    CBFM_REQUIRE(prm->gen_host && prm->n_gen > 0, CBFM_E_ARG, "need generating waves");
    CBFM_REQUIRE(prm->delta_svd >= 0 && prm->delta_svd <= 1, CBFM_E_ARG, "delta_svd outside [0, 1]");
    const Media md = make_media(med);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MeshHost& h = m->h;
    const int nb = h.nblocks;
    const int S = prm->n_gen;
    int Nmax = 0;
    for (int b = 0; b < nb; ++b) Nmax = std::max<int>(Nmax, (int)(h.cell_off[b + 1] - h.cell_off[b]));
    const int n = 2 * Nmax;
    // generating right-hand sides on all edges
    Scratch vgen((size_t)S * 2 * h.ne * sizeof(double2), s);
    Scratch dinc((size_t)S * 6 * sizeof(double), s);
    CBFM_HIP(hipMemcpyAsync(dinc.p, prm->gen_host, (size_t)S * 6 * sizeof(double), hipMemcpyHostToDevice, s));
    rhs_launch(m, md, med->eta0, dinc.as<double>(), S, vgen.p, s);
    // per-cell Z_mm (padded, column-major) and V_m
    Scratch Zpad((size_t)nb * n * n * sizeof(double2), s);
    Scratch Vpad((size_t)nb * n * S * sizeof(double2), s);
    Scratch ops((size_t)3 * Nmax * Nmax * sizeof(double2), s);
    // index staging for every cell, uploaded once
    std::vector<CellSupport> cs(nb);
    size_t ibytes = 0;
    for (int b = 0; b < nb; ++b) {
      cs[b] = support(h, cell_edges(h, b));
      ibytes += 4 * (cs[b].tris.size() + cs[b].pos.size() + cs[b].edges.size()) + sizeof(NearPair) * cs[b].near.size();
    }
    std::vector<char> host(ibytes);
    Scratch idx(ibytes, s);
    size_t o = 0;
    struct Ptrs {
      int32_t *tris, *pos, *edges;
      NearPair* near;
    };
    std::vector<Ptrs> ptr(nb);
    auto put = [&](const void* src, size_t bytes) {
      std::memcpy(host.data() + o, src, bytes);
      void* d = idx.as<char>() + o;
      o += bytes;
      return d;
    };
    size_t maxloc = 0;
    for (int b = 0; b < nb; ++b) {
      ptr[b].tris = (int32_t*)put(cs[b].tris.data(), 4 * cs[b].tris.size());
      ptr[b].pos = (int32_t*)put(cs[b].pos.data(), 4 * cs[b].pos.size());
      ptr[b].edges = (int32_t*)put(cs[b].edges.data(), 4 * cs[b].edges.size());
      ptr[b].near = (NearPair*)put(cs[b].near.data(), sizeof(NearPair) * cs[b].near.size());
      maxloc = std::max(maxloc, cs[b].tris.size());
    }
    CBFM_HIP(hipMemcpyAsync(idx.p, host.data(), ibytes, hipMemcpyHostToDevice, s));
    Scratch local((size_t)27 * maxloc * maxloc * sizeof(double2), s);
    for (int b = 0; b < nb; ++b) {
      const int Nb = (int)cs[b].edges.size();
      const int64_t nt_b = cs[b].tris.size();
      fill_local(m, md, CBFM_FP64, CBFM_LAYOUT_OPS3, ptr[b].tris, nt_b, ptr[b].tris, nt_b, ptr[b].near,
                 (int64_t)cs[b].near.size(), local.p, s);
      assemble(m, CBFM_FP64, local.p, nt_b, nt_b, ptr[b].edges, Nb, ptr[b].edges, Nb, ptr[b].pos, ptr[b].pos, ops.p,
               (int64_t)Nb * Nb, Nb, s);
      double2* Zb = Zpad.as<double2>() + (size_t)b * n * n;
      hipLaunchKernelGGL(pack_zmm_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, ops.as<double2>(), Nb, n, Zb);
      hipLaunchKernelGGL(pack_v_kernel, dim3((n + 255) / 256, S), dim3(256), 0, s, vgen.as<double2>(), h.ne,
                         ptr[b].edges, Nb, n, Vpad.as<double2>() + (size_t)b * n * S);
      CBFM_HIP(hipGetLastError());
    }
    // LU solves Z_mm J_m = V_m
    Scratch piv((size_t)nb * n * sizeof(rocblas_int), s);
    Scratch info((size_t)nb * sizeof(rocblas_int), s);
    {
      std::lock_guard<std::mutex> lk(blas_mutex());
      rocblas_handle bh = blas_handle(s);
      CBFM_RS(rocsolver_zgetrf_strided_batched(bh, n, n, (rocblas_double_complex*)Zpad.p, n, (rocblas_stride)n * n,
                                               piv.as<rocblas_int>(), n, info.as<rocblas_int>(), nb));
      CBFM_RS(rocsolver_zgetrs_strided_batched(bh, rocblas_operation_none, n, S, (rocblas_double_complex*)Zpad.p, n,
                                               (rocblas_stride)n * n, piv.as<rocblas_int>(), n,
                                               (rocblas_double_complex*)Vpad.p, n, (rocblas_stride)n * S, nb));
    }
    std::vector<rocblas_int> hinfo(nb);
    CBFM_HIP(hipMemcpyAsync(hinfo.data(), info.p, nb * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    CBFM_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
      CBFM_REQUIRE(hinfo[b] == 0, CBFM_E_RANK, "cell " + std::to_string(b) + ": Z_mm is singular");
    // QR of (J^M)^H and (J^J)^H (column-major S x Nmax, zero-padded)
    const int rk = std::min(S, Nmax);
    Scratch QA((size_t)nb * 2 * S * Nmax * sizeof(double2), s);
    Scratch tau((size_t)nb * 2 * rk * sizeof(double2), s);
    for (int b = 0; b < nb; ++b) {
      const int Nb = (int)cs[b].edges.size();
      hipLaunchKernelGGL(pack_jh_kernel, dim3((S + 255) / 256, Nmax, 2), dim3(256), 0, s,
                         Vpad.as<double2>() + (size_t)b * n * S, n, S, Nb, Nmax,
                         QA.as<double2>() + (size_t)b * 2 * S * Nmax);
    }
    CBFM_HIP(hipGetLastError());
    {
      std::lock_guard<std::mutex> lk(blas_mutex());
      rocblas_handle bh = blas_handle(s);
      CBFM_RS(rocsolver_zgeqrf_strided_batched(bh, S, Nmax, (rocblas_double_complex*)QA.p, S,
                                               (rocblas_stride)S * Nmax, (rocblas_double_complex*)tau.p,
                                               (rocblas_stride)rk, 2 * nb));
    }
    // R factors (row-major rk x Nmax) and the core X = C^T, C = R_M G_m R_J^H
    // (G_m real antisymmetric: X = conj(R_J) G_m^T R_M^T = -conj(R_J) G_m R_M^T)
    Scratch Rf((size_t)nb * 2 * rk * Nmax * sizeof(double2), s);
    Scratch Gm((size_t)nb * Nmax * Nmax * sizeof(double2), s);
    Scratch T2((size_t)nb * Nmax * rk * sizeof(double2), s);
    Scratch core((size_t)nb * rk * rk * sizeof(double2), s);
    std::vector<GemmDesc> d1, d2;
    for (int b = 0; b < nb; ++b) {
      const int Nb = (int)cs[b].edges.size();
      double2* R = Rf.as<double2>() + (size_t)b * 2 * rk * Nmax;  // R_M, then R_J
      hipLaunchKernelGGL(extract_r_kernel, dim3((Nmax + 255) / 256, rk, 2), dim3(256), 0, s,
                         QA.as<double2>() + (size_t)b * 2 * S * Nmax, S, Nb, Nmax, rk, R);
      double2* G = Gm.as<double2>() + (size_t)b * Nmax * Nmax;
      hipLaunchKernelGGL(cell_gram_kernel, dim3((Nb + 255) / 256, Nb), dim3(256), 0, s, ptr[b].edges, Nb,
                         m->tplus.as<int32_t>(), m->tminus.as<int32_t>(), m->aplus.as<int32_t>(),
                         m->aminus.as<int32_t>(), m->tri_edge.as<int32_t>(), m->tri_sign.as<int32_t>(),
                         m->length.as<double>(), G);
      double2* t2 = T2.as<double2>() + (size_t)b * Nmax * rk;
      d1.push_back(gemm(G, Nb, OP_N, R, Nmax, OP_T, t2, rk, Nb, rk, Nb));
      d2.push_back(gemm(R + (size_t)rk * Nmax, Nmax, OP_R, t2, rk, OP_N, core.as<double2>() + (size_t)b * rk * rk, rk,
                        rk, rk, Nb, -1.0));
    }
    CBFM_HIP(hipGetLastError());
    zgemm_batched(d1, s);
    zgemm_batched(d2, s);
    // SVD of the cores
    Scratch sv((size_t)nb * rk * sizeof(double), s);
    Scratch U((size_t)nb * rk * rk * sizeof(double2), s);
    Scratch Vh((size_t)nb * rk * rk * sizeof(double2), s);
    Scratch E((size_t)nb * rk * sizeof(double), s);
    {
      std::lock_guard<std::mutex> lk(blas_mutex());
      rocblas_handle bh = blas_handle(s);
      CBFM_RS(rocsolver_zgesvd_strided_batched(
          bh, rocblas_svect_singular, rocblas_svect_singular, rk, rk, (rocblas_double_complex*)core.p, rk,
          (rocblas_stride)rk * rk, sv.as<double>(), rk, (rocblas_double_complex*)U.p, rk, (rocblas_stride)rk * rk,
          (rocblas_double_complex*)Vh.p, rk, (rocblas_stride)rk * rk, E.as<double>(), rk, rocblas_outofplace,
          info.as<rocblas_int>(), nb));
    }
    std::vector<double> hs((size_t)nb * rk);
    CBFM_HIP(hipMemcpyAsync(hs.data(), sv.p, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CBFM_HIP(hipMemcpyAsync(hinfo.data(), info.p, nb * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    CBFM_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
      CBFM_REQUIRE(hinfo[b] == 0, CBFM_E_HIP, "cell " + std::to_string(b) + ": SVD did not converge");
    auto* c = new cbfm_cbf_s();
    try {
      c->mesh = m;
      c->L.resize(nb);
      for (int b = 0; b < nb; ++b) {
        const double* sb = &hs[(size_t)b * rk];
        int L = 0;
        const int Nb = (int)cs[b].edges.size();
        while (L < rk && L < Nb && sb[L] > 0 && sb[L] >= prm->delta_svd * sb[0]) ++L;
        if (prm->max_L > 0) L = std::min(L, prm->max_L);
        CBFM_REQUIRE(L > 0, CBFM_E_RANK, "cell " + std::to_string(b) + " keeps no CBF");
        c->L[b] = L;
        c->sigma.insert(c->sigma.end(), sb, sb + L);
      }
      cbf_finish(c);
      c->CM.alloc(std::max<int64_t>(1, c->coff[nb]) * sizeof(double2));
      c->CJ.alloc(std::max<int64_t>(1, c->coff[nb]) * sizeof(double2));
      // C^M = R_M^H U_c,L and C^J = R_J^H V_c,L (U_c column-major, V_c^H column-major)
      std::vector<GemmDesc> d3;
      for (int b = 0; b < nb; ++b) {
        const int Nb = (int)cs[b].edges.size();
        const double2* R = Rf.as<double2>() + (size_t)b * 2 * rk * Nmax;
        d3.push_back(gemm(R, Nmax, OP_C, U.as<double2>() + (size_t)b * rk * rk, rk, OP_T,
                          c->CM.as<double2>() + c->coff[b], c->L[b], Nb, c->L[b], rk));
        d3.push_back(gemm(R + (size_t)rk * Nmax, Nmax, OP_C, Vh.as<double2>() + (size_t)b * rk * rk, rk, OP_R,
                          c->CJ.as<double2>() + c->coff[b], c->L[b], Nb, c->L[b], rk));
      }
      zgemm_batched(d3, s);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

cbfm_status cbfm_cbf_import(cbfm_mesh m, const int32_t* L, const void* CM, const void* CJ, const double* sigma,
                            void* stream, cbfm_cbf* out) {
  return guarded([&] {
    CBFM_REQUIRE(m && L && CM && CJ && sigma && out, CBFM_E_ARG, "null argument");
    *out = nullptr;
    const MeshHost& h = m->h;
    auto* c = new cbfm_cbf_s();
    try {
      c->mesh = m;
      c->L.assign(L, L + h.nblocks);
      for (int b = 0; b < h.nblocks; ++b) {
        const int64_t Nb = h.cell_off[b + 1] - h.cell_off[b];
        CBFM_REQUIRE(c->L[b] > 0 && c->L[b] <= Nb, CBFM_E_ARG, "L out of range for cell " + std::to_string(b));
      }
      cbf_finish(c);
      c->sigma.assign(sigma, sigma + c->NL);
      const size_t bytes = c->coff[h.nblocks] * sizeof(double2);
      c->CM.alloc(bytes);
      c->CJ.alloc(bytes);
      CBFM_HIP(hipMemcpy(c->CM.p, CM, bytes, hipMemcpyHostToDevice));
      CBFM_HIP(hipMemcpy(c->CJ.p, CJ, bytes, hipMemcpyHostToDevice));
      (void)stream;
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

cbfm_status cbfm_cbf_info(cbfm_cbf c, int64_t* n_cbf, int32_t* L, double* sigma) {
  return guarded([&] {
    CBFM_REQUIRE(c != nullptr, CBFM_E_ARG, "cbf is NULL");
    if (n_cbf) *n_cbf = 2 * c->NL;
    if (L) std::memcpy(L, c->L.data(), c->L.size() * sizeof(int32_t));
    if (sigma) std::memcpy(sigma, c->sigma.data(), c->sigma.size() * sizeof(double));
  });
}

cbfm_status cbfm_cbf_export(cbfm_cbf c, void* CM, void* CJ) {
  return guarded([&] {
    CBFM_REQUIRE(c != nullptr, CBFM_E_ARG, "cbf is NULL");
    const size_t bytes = c->coff.back() * sizeof(double2);
    if (CM) CBFM_HIP(hipMemcpy(CM, c->CM.p, bytes, hipMemcpyDeviceToHost));
    if (CJ) CBFM_HIP(hipMemcpy(CJ, c->CJ.p, bytes, hipMemcpyDeviceToHost));
  });
}

void cbfm_cbf_free(cbfm_cbf c) { delete c; }

cbfm_status cbfm_cmp_apply(cbfm_cbf c, int64_t nrhs, const void* y, void* x, void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(c && y && x && nrhs >= 0, CBFM_E_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (x != y)
      CBFM_HIP(hipMemcpyAsync(x, y, (size_t)nrhs * 2 * c->NL * sizeof(double2), hipMemcpyDeviceToDevice, s));
    cmp_apply_dev(c, nrhs, static_cast<double2*>(x), s);
  });
}

}  // extern "C"
