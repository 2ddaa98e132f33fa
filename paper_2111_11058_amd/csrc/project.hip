// Reduced matrix Z_r = (C^JM)^H Z C^MJ (paper Sec. III-C, outer CBFM
// equation), with Z = [[K, -TE], [TH, K]]:
//   Z_r = [[ (C^J)^H K C^M, -(C^J)^H TE C^J ],
//          [ (C^M)^H TH C^M,  (C^M)^H K C^J ]]
// Rows are processed in panels of whole cells.  For a panel the fill
// kernels produce the triangle-local blocks of the panel's test triangles
// against every source triangle, the gather kernel assembles the panel's
// rows of K, TE, TH (upcast to double, or kept in float for the mixed
// forms), and two batched matrix-core GEMM launches (FP64, or FP32 / BF16
// inputs with FP32 accumulation) form
//   W_X[rows, cell b] = X[rows, cell b] C_b          (X in K, TE, TH)
//   Z_r[cell a rows]  = C_a^H W_X[cell a rows, :]
// so only one panel of Z exists at a time.
#include <algorithm>
#include <cstring>

#include "cbf.h"
#include "gemm.h"

namespace cbfm {

// Bytes of scratch a panel of `nrow` RWG rows touching `nrt` triangles needs.
static size_t panel_bytes(int64_t nrt, int64_t nt, int64_t nrow, int64_t ne, int64_t NL, size_t esz) {
  return (size_t)27 * nrt * nt * esz + (size_t)3 * nrow * ne * 16 + (size_t)4 * nrow * NL * 16;
}

void project_dev(const cbfm_mesh_s* m, const Media& md, cbfm_cbf_s* c, int precision, double2* Zr, int64_t ldz,
                 hipStream_t s, size_t budget) {
  const MeshHost& h = m->h;
  const int nb = h.nblocks;
  const int64_t ne = h.ne, nt = h.nt, NL = c->NL;
  // mixed forms: FP32 regular fill, panel and W in complex float, projection
  // on the FP32 or BF16 matrix cores (FP32 accumulation), Z_r stored double
  const bool mixed = precision == CBFM_MIXED_FP32 || precision == CBFM_MIXED_BF16 || precision == CBFM_MIXED_BF16X3;
  const int fillp = precision == CBFM_FP64 ? CBFM_FP64 : CBFM_FP32;
  const size_t esz = fillp == CBFM_FP64 ? 16 : 8;
  // column side: every triangle, every edge (internal order)
  std::vector<int32_t> iota(nt);
  for (int64_t t = 0; t < nt; ++t) iota[t] = (int32_t)t;
  // group cells into panels whose scratch fits the budget
  std::vector<int32_t> mark(nt, -1);
  int a0 = 0;
  std::vector<std::pair<int, int>> panels;
  while (a0 < nb) {
    int a1 = a0;
    int64_t nrt = 0;
    int stamp = a0;
    while (a1 < nb) {
      // triangles of cells a0..a1
      int64_t add = 0;
      for (int64_t i = h.cell_off[a1]; i < h.cell_off[a1 + 1]; ++i) {
        const int e = h.perm[i];
        for (int t : {h.tplus[e], h.tminus[e]})
          if (mark[t] != stamp) {
            mark[t] = stamp;
            ++add;
          }
      }
      const int64_t nrow = h.cell_off[a1 + 1] - h.cell_off[a0];
      // (marks carry the panel's first cell as stamp, so the next panel recounts)
      if (a1 > a0 && panel_bytes(nrt + add, nt, nrow, ne, NL, esz) > budget) break;
      nrt += add;
      ++a1;
    }
    panels.push_back({a0, a1});
    a0 = a1;
  }
  // device index tables shared by all panels
  Scratch dcol((size_t)(2 * nt) * sizeof(int32_t), s);
  CBFM_HIP(hipMemcpyAsync(dcol.p, iota.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, s));
  CBFM_HIP(hipMemcpyAsync(dcol.as<int32_t>() + nt, iota.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, s));
  const int32_t* colTris = dcol.as<int32_t>();
  const int32_t* colPos = dcol.as<int32_t>() + nt;
  const int32_t* colEdges = m->perm.as<int32_t>();

  for (auto [p0, p1] : panels) {
    const int64_t r0 = h.cell_off[p0], nrow = h.cell_off[p1] - r0;
    std::vector<int32_t> pos(nt, -1), rows, redges(h.perm.begin() + r0, h.perm.begin() + r0 + nrow);
    for (int e : redges) {
      pos[h.tplus[e]] = 0;
      pos[h.tminus[e]] = 0;
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
    const size_t ib = 4 * (rows.size() + pos.size() + redges.size()) + sizeof(NearPair) * nl.size();
    std::vector<char> host(ib);
    Scratch idx(ib, s);
    size_t o = 0;
    auto put = [&](const void* src, size_t bytes) {
      std::memcpy(host.data() + o, src, bytes);
      void* d = idx.as<char>() + o;
      o += bytes;
      return d;
    };
    auto* d_rows = (int32_t*)put(rows.data(), 4 * rows.size());
    auto* d_pos = (int32_t*)put(pos.data(), 4 * pos.size());
    auto* d_re = (int32_t*)put(redges.data(), 4 * redges.size());
    auto* d_nl = (NearPair*)put(nl.data(), sizeof(NearPair) * nl.size());
    CBFM_HIP(hipMemcpyAsync(idx.p, host.data(), ib, hipMemcpyHostToDevice, s));
    Scratch local((size_t)27 * nrt * nt * esz, s);
    const size_t zsz = mixed ? sizeof(float2) : sizeof(double2);
    Scratch Zp((size_t)3 * nrow * ne * zsz, s);
    Scratch W((size_t)4 * nrow * NL * zsz, s);
    fill_local(m, md, fillp, CBFM_LAYOUT_OPS3, d_rows, nrt, colTris, nt, d_nl, (int64_t)nl.size(), local.p, s);
    assemble(m, fillp, local.p, nrt, nt, d_re, nrow, colEdges, ne, d_pos, colPos, Zp.p, nrow * ne, ne, s,
             mixed ? 0 : 1);
    if (mixed) {
      const float2* Zk = Zp.as<float2>();
      const float2* Zte = Zk + nrow * ne;
      const float2* Zth = Zte + nrow * ne;
      float2* Wkm = W.as<float2>();
      float2* Wkj = Wkm + nrow * NL;
      float2* Wte = Wkj + nrow * NL;
      float2* Wth = Wte + nrow * NL;
      std::vector<GemmDescX> x1, x2;
      for (int b = 0; b < nb; ++b) {
        const int64_t Nb = h.cell_off[b + 1] - h.cell_off[b], cb0 = h.cell_off[b];
        const double2* CMb = c->CM.as<double2>() + c->coff[b];
        const double2* CJb = c->CJ.as<double2>() + c->coff[b];
        const int64_t Lb = c->L[b], ob = c->off[b];
        x1.push_back(gemmx(Zk + cb0, 0, ne, OP_N, CMb, 1, Lb, OP_N, Wkm + ob, 0, NL, nrow, Lb, Nb));
        x1.push_back(gemmx(Zk + cb0, 0, ne, OP_N, CJb, 1, Lb, OP_N, Wkj + ob, 0, NL, nrow, Lb, Nb));
        x1.push_back(gemmx(Zte + cb0, 0, ne, OP_N, CJb, 1, Lb, OP_N, Wte + ob, 0, NL, nrow, Lb, Nb));
        x1.push_back(gemmx(Zth + cb0, 0, ne, OP_N, CMb, 1, Lb, OP_N, Wth + ob, 0, NL, nrow, Lb, Nb));
      }
      for (int a = p0; a < p1; ++a) {
        const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], ra = h.cell_off[a] - r0;
        const double2* CMa = c->CM.as<double2>() + c->coff[a];
        const double2* CJa = c->CJ.as<double2>() + c->coff[a];
        const int64_t La = c->L[a], oa = c->off[a];
        x2.push_back(gemmx(CJa, 1, La, OP_C, Wkm + ra * NL, 0, NL, OP_N, Zr + oa * ldz, 1, ldz, La, NL, Na));
        x2.push_back(gemmx(CJa, 1, La, OP_C, Wte + ra * NL, 0, NL, OP_N, Zr + oa * ldz + NL, 1, ldz, La, NL, Na, -1.0f));
        x2.push_back(gemmx(CMa, 1, La, OP_C, Wth + ra * NL, 0, NL, OP_N, Zr + (NL + oa) * ldz, 1, ldz, La, NL, Na));
        x2.push_back(gemmx(CMa, 1, La, OP_C, Wkj + ra * NL, 0, NL, OP_N, Zr + (NL + oa) * ldz + NL, 1, ldz, La, NL, Na));
      }
      const int mode = precision == CBFM_MIXED_BF16 ? XG_BF16 : precision == CBFM_MIXED_BF16X3 ? XG_BF16X3 : XG_FP32;
      xgemm_batched(x1, mode, s);
      xgemm_batched(x2, mode, s);
      continue;  // xgemm_batched synchronised the stream
    }
    double2* Zk = Zp.as<double2>();
    double2* Zte = Zk + nrow * ne;
    double2* Zth = Zte + nrow * ne;
    double2* Wkm = W.as<double2>();
    double2* Wkj = Wkm + nrow * NL;
    double2* Wte = Wkj + nrow * NL;
    double2* Wth = Wte + nrow * NL;
    std::vector<GemmDesc> d1, d2;
    for (int b = 0; b < nb; ++b) {
      const int64_t Nb = h.cell_off[b + 1] - h.cell_off[b], cb0 = h.cell_off[b];
      const double2* CMb = c->CM.as<double2>() + c->coff[b];
      const double2* CJb = c->CJ.as<double2>() + c->coff[b];
      const int64_t Lb = c->L[b], ob = c->off[b];
      d1.push_back(gemm(Zk + cb0, ne, OP_N, CMb, Lb, OP_N, Wkm + ob, NL, nrow, Lb, Nb));
      d1.push_back(gemm(Zk + cb0, ne, OP_N, CJb, Lb, OP_N, Wkj + ob, NL, nrow, Lb, Nb));
      d1.push_back(gemm(Zte + cb0, ne, OP_N, CJb, Lb, OP_N, Wte + ob, NL, nrow, Lb, Nb));
      d1.push_back(gemm(Zth + cb0, ne, OP_N, CMb, Lb, OP_N, Wth + ob, NL, nrow, Lb, Nb));
    }
    for (int a = p0; a < p1; ++a) {
      const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], ra = h.cell_off[a] - r0;
      const double2* CMa = c->CM.as<double2>() + c->coff[a];
      const double2* CJa = c->CJ.as<double2>() + c->coff[a];
      const int64_t La = c->L[a], oa = c->off[a];
      d2.push_back(gemm(CJa, La, OP_C, Wkm + ra * NL, NL, OP_N, Zr + oa * ldz, ldz, La, NL, Na));
      d2.push_back(gemm(CJa, La, OP_C, Wte + ra * NL, NL, OP_N, Zr + oa * ldz + NL, ldz, La, NL, Na, -1.0));
      d2.push_back(gemm(CMa, La, OP_C, Wth + ra * NL, NL, OP_N, Zr + (NL + oa) * ldz, ldz, La, NL, Na));
      d2.push_back(gemm(CMa, La, OP_C, Wkj + ra * NL, NL, OP_N, Zr + (NL + oa) * ldz + NL, ldz, La, NL, Na));
    }
    zgemm_batched(d1, s);
    zgemm_batched(d2, s);
    CBFM_HIP(hipStreamSynchronize(s));  // host index staging of this panel
  }
}

}  // namespace cbfm

using namespace cbfm;

extern "C" cbfm_status cbfm_project(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, int32_t precision, void* Zr,
                                    int64_t ldz, void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(m && c && Zr, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(c->mesh == m, CBFM_E_STATE, "CBF set belongs to another mesh");
    CBFM_REQUIRE(precision == CBFM_FP64 || precision == CBFM_FP32 || precision == CBFM_MIXED_FP32 ||
                     precision == CBFM_MIXED_BF16 || precision == CBFM_MIXED_BF16X3,
                 CBFM_E_ARG, "unknown precision");
    CBFM_REQUIRE(ldz >= 2 * c->NL, CBFM_E_ARG, "ldz < N_CBF");
    const Media md = make_media(med);
    // scratch budget per panel: a quarter of the free device memory, at most 32 GiB
    size_t fr = 0, tot = 0;
    CBFM_HIP(hipMemGetInfo(&fr, &tot));
    const size_t budget = std::min<size_t>(fr / 4, (size_t)32 << 30);
    project_dev(m, md, c, precision, static_cast<double2*>(Zr), ldz, static_cast<hipStream_t>(stream), budget);
  });
}
