// Reduced matrix Z_r = (C^JM)^H Z C^MJ (paper Sec. III-C, outer CBFM
// equation), with Z = [[K, -TE], [TH, K]]:
//   Z_r = [[ (C^J)^H K C^M, -(C^J)^H TE C^J ],
//          [ (C^M)^H TH C^M,  (C^M)^H K C^J ]]
// Rows are processed in panels of whole cells.  For a panel the fill
// kernels produce the triangle-local blocks of the panel's test triangles
// against the source triangles of its own and the later cells (the rest
// follows by reciprocity, below), the gather kernel assembles blocks of
// K, TE, TH (upcast to double, or kept in float for the mixed forms), and
// two batched matrix-core GEMM launches per block (FP64, or FP32 / BF16
// inputs with FP32 accumulation) form
//   W_X[rows, cell b] = X[rows, cell b] C_b          (X in K, TE, TH)
//   Z_r[cell a rows]  = C_a^H W_X[cell a rows, :]
// so only one panel of Z exists at a time.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>

#include "cbf.h"
#include "gemm.h"

namespace cbfm {

// Descriptors of the projection GEMMs of one block of Z: the rows of cells
// ra0..ra1-1 against the columns of cells cb0..cb1-1.  Zp holds [K; TE; TH]
// of the block (complex float for the mixed forms, else double), each
// plane nrow x ncol row-major with leading dimension zld, or stored
// transposed (ncol x nrow, trans) as the reversed block; W receives the
// four nrow x NLc products (NLc = CBFs of the column cells).  plane: the
// elements from one operator's plane to the next (0: nrow x ncol).
static void block_gemms(const MeshHost& h, cbfm_cbf_s* c, int ra0, int ra1, int cb0, int cb1, void* Zp, int64_t zld,
                        bool trans, void* W, bool mixed, double2* Zr, int64_t ldz, std::vector<GemmDesc>& d1,
                        std::vector<GemmDesc>& d2, std::vector<GemmDescX>& x1, std::vector<GemmDescX>& x2,
                        int64_t plane = 0) {
  const int64_t NL = c->NL, r0 = h.cell_off[ra0], nrow = h.cell_off[ra1] - r0;
  const int64_t c0 = h.cell_off[cb0], ncol = h.cell_off[cb1] - c0;
  const int64_t o0 = c->off[cb0], NLc = c->off[cb1] - o0;
  const size_t zs = mixed ? sizeof(float2) : sizeof(double2);
  const int64_t zplane = plane > 0 ? plane : nrow * ncol;  // elements between the K, TE, TH planes
  char* Zk = static_cast<char*>(Zp);
  char* Zte = Zk + zplane * zs;
  char* Zth = Zte + zplane * zs;
  char* Wkm = static_cast<char*>(W);
  char* Wkj = Wkm + nrow * NLc * zs;
  char* Wte = Wkj + nrow * NLc * zs;
  char* Wth = Wte + nrow * NLc * zs;
  const int opZ = trans ? OP_T : OP_N;
  for (int b = cb0; b < cb1; ++b) {
    const int64_t Nb = h.cell_off[b + 1] - h.cell_off[b], cb = h.cell_off[b] - c0;
    const int64_t zoff = trans ? cb * zld : cb;  // cell b's columns of the block
    const double2* CMb = c->CM.as<double2>() + c->coff[b];
    const double2* CJb = c->CJ.as<double2>() + c->coff[b];
    const int64_t Lb = c->L[b], ob = c->off[b] - o0;
    const struct {
      char* Z;
      const double2* C;
      char* W;
    } prod[4] = {{Zk, CMb, Wkm}, {Zk, CJb, Wkj}, {Zte, CJb, Wte}, {Zth, CMb, Wth}};
    for (const auto& q : prod) {
      if (mixed)
        x1.push_back(gemmx(q.Z + zoff * zs, 0, zld, opZ, q.C, 1, Lb, OP_N, q.W + ob * zs, 0, NLc, nrow, Lb, Nb));
      else
        d1.push_back(gemm(reinterpret_cast<const double2*>(q.Z) + zoff, zld, opZ, q.C, Lb, OP_N,
                          reinterpret_cast<double2*>(q.W) + ob, NLc, nrow, Lb, Nb));
    }
  }
  for (int a = ra0; a < ra1; ++a) {
    const int64_t Na = h.cell_off[a + 1] - h.cell_off[a], ra = h.cell_off[a] - r0;
    const double2* CMa = c->CM.as<double2>() + c->coff[a];
    const double2* CJa = c->CJ.as<double2>() + c->coff[a];
    const int64_t La = c->L[a], oa = c->off[a];
    // Z_r blocks: [J rows][M cols] = C^J^H K C^M, [J][J] = -C^J^H TE C^J,
    //             [M][M] = C^M^H TH C^M,         [M][J] = C^M^H K C^J
    const struct {
      const double2* C;
      char* W;
      double2* out;
      double alpha;
    } prod[4] = {{CJa, Wkm, Zr + oa * ldz + o0, 1.0},
                 {CJa, Wte, Zr + oa * ldz + NL + o0, -1.0},
                 {CMa, Wth, Zr + (NL + oa) * ldz + o0, 1.0},
                 {CMa, Wkj, Zr + (NL + oa) * ldz + NL + o0, 1.0}};
    for (const auto& q : prod) {
      if (mixed)
        x2.push_back(gemmx(q.C, 1, La, OP_C, q.W + ra * NLc * zs, 0, NLc, OP_N, q.out, 1, ldz, La, NLc, Na,
                           (float)q.alpha));
      else
        d2.push_back(gemm(q.C, La, OP_C, reinterpret_cast<const double2*>(q.W) + ra * NLc, NLc, OP_N, q.out, ldz, La,
                          NLc, Na, q.alpha));
    }
  }
}

// The rows of cells p0..p1-1 against every column (one whole block row).
static void panel_gemms(const MeshHost& h, cbfm_cbf_s* c, int p0, int p1, void* Zp, void* W, bool mixed, double2* Zr,
                        int64_t ldz, std::vector<GemmDesc>& d1, std::vector<GemmDesc>& d2, std::vector<GemmDescX>& x1,
                        std::vector<GemmDescX>& x2) {
  block_gemms(h, c, p0, p1, 0, h.nblocks, Zp, h.ne, false, W, mixed, Zr, ldz, d1, d2, x1, x2);
}

// Both GEMM stages (each one batched launch; both synchronise the stream).
// (with keepd / keepx the staged descriptors stay with the caller, which
// synchronises s before releasing them; otherwise each launch synchronises)
static void launch_panel_gemms(int precision, std::vector<GemmDesc>& d1, std::vector<GemmDesc>& d2,
                               std::vector<GemmDescX>& x1, std::vector<GemmDescX>& x2, hipStream_t s,
                               std::vector<std::vector<GemmDesc>>* keepd = nullptr,
                               std::vector<std::vector<GemmDescX>>* keepx = nullptr) {
  const int mode = precision == CBFM_MIXED_BF16 ? XG_BF16 : precision == CBFM_MIXED_BF16X3 ? XG_BF16X3 : XG_FP32;
  if (!x1.empty()) {
    xgemm_batched(x1, mode, s, keepx);
    xgemm_batched(x2, mode, s, keepx);
  }
  if (!d1.empty()) {
    zgemm_batched(d1, s, keepd);
    zgemm_batched(d2, s, keepd);
  }
}

// Reciprocity: for the regular rule every operator's triangle-local block
// of (test P, source Q) is the transpose of that of (Q, P) (the integrands
// of T_i and of K agree point by point under the exchange; Sec. II-B), and
// the near-pair rule is evaluated in both orientations.  Panel p (row
// cells p0..p1-1) therefore fills its test triangles only against the
// source triangles of cells p0..nb-1 and yields two blocks of Z:
//   the block row  Z[cells p0..p1-1][cells p0..nb-1], and, after the near
//   pairs of the later cells' triangles (test) against the panel's
//   (source) are written over their reversed slots,
//   the block column Z[cells p1..nb-1][cells p0..p1-1], assembled from the
//   same local blocks as its transpose.
// The block column stored transposed is the block row's later-cell part,
// except where a triangle pair of the entry is a near pair: so it is not
// assembled again; only those entries of the block row's storage are
// re-gathered after the reversed near values are written (once the block
// row's GEMMs have read it), and the block column's GEMMs read the same
// storage.
// Every block of Z_r comes from exactly one of them.  With panels of an
// eighth of the cells about 9/16 of the regular pairs are computed.
static size_t panel_bytes(int64_t nrt, int64_t nct, int64_t nrow, int64_t ncol, int64_t nlater, int64_t NLc,
                          int64_t NLp, size_t esz, size_t zs) {
  return (size_t)27 * nrt * nct * esz + (size_t)3 * nrow * ncol * zs +
         std::max((size_t)4 * nrow * NLc, (size_t)4 * nlater * NLp) * zs;
}

int project_dev(const cbfm_mesh_s* m, const Media& md, cbfm_cbf_s* c, int precision, double2* Zr, int64_t ldz,
                hipStream_t s, size_t budget) {
  const MeshHost& h = m->h;
  const int nb = h.nblocks;
  const int64_t ne = h.ne, nt = h.nt;
  // mixed forms: FP32 regular fill, panel and W in complex float, projection
  // on the FP32 or BF16 matrix cores (FP32 accumulation), Z_r stored double
  const bool mixed = precision == CBFM_MIXED_FP32 || precision == CBFM_MIXED_BF16 || precision == CBFM_MIXED_BF16X3;
  const int fillp = precision == CBFM_FP64 ? CBFM_FP64 : CBFM_FP32;
  const size_t esz = fillp == CBFM_FP64 ? 16 : 8;
  const size_t zs = mixed ? sizeof(float2) : sizeof(double2);
  // triangles of each cell's RWGs, and how many cells from a0 on touch each
  // triangle's support (for the column triangle counts)
  std::vector<std::vector<int32_t>> ctris(nb);
  {
    std::vector<int32_t> mark(nt, -1);
    for (int b = 0; b < nb; ++b)
      for (int64_t i = h.cell_off[b]; i < h.cell_off[b + 1]; ++i) {
        const int e = h.perm[i];
        for (int t : {h.tplus[e], h.tminus[e]})
          if (mark[t] != b) {
            mark[t] = b;
            ctris[b].push_back(t);
          }
      }
  }
  // nct(a0): triangles of the RWGs of cells a0..nb-1
  std::vector<int64_t> nct_from(nb + 1, 0);
  {
    std::vector<char> seen(nt, 0);
    for (int b = nb - 1; b >= 0; --b) {
      int64_t add = 0;
      for (int t : ctris[b])
        if (!seen[t]) {
          seen[t] = 1;
          ++add;
        }
      nct_from[b] = nct_from[b + 1] + add;
    }
  }
  // panels of consecutive cells, within the budget; on meshes of 4,096
  // triangles or more at most ceil(nb / 8) cells each, so that reciprocity
  // saves about 7/16 of the regular pairs (on smaller meshes the fixed cost
  // of a panel outweighs it: one panel when the budget allows)
  const int max_cells = nt >= 4096 ? std::max(1, (nb + 7) / 8) : nb;
  std::vector<std::pair<int, int>> panels;
  {
    std::vector<int32_t> mark(nt, -1);
    int a0 = 0;
    while (a0 < nb) {
      int a1 = a0;
      int64_t nrt = 0;
      while (a1 < nb && a1 - a0 < max_cells) {
        int64_t add = 0;
        for (int t : ctris[a1])
          if (mark[t] != a0) {
            mark[t] = a0;
            ++add;
          }
        const int64_t nrow = h.cell_off[a1 + 1] - h.cell_off[a0];
        const size_t need = panel_bytes(nrt + add, nct_from[a0], nrow, ne - h.cell_off[a0], ne - h.cell_off[a1 + 1],
                                        c->NL - c->off[a0], c->off[a1 + 1] - c->off[a0], esz, zs);
        if (a1 > a0 && need > budget) break;
        nrt += add;
        ++a1;
      }
      panels.push_back({a0, a1});
      a0 = a1;
    }
  }

  // The panels are queued without waiting for one another: the host
  // prepares the next panel's index tables while the device works on this
  // one.  Staged host data (index tables, GEMM descriptors) is kept until
  // the final synchronisation.
  std::vector<std::vector<char>> staged;
  std::vector<std::vector<GemmDesc>> keepd;
  std::vector<std::vector<GemmDescX>> keepx;
  for (auto [p0, p1] : panels) {
    const int64_t r0 = h.cell_off[p0], r1 = h.cell_off[p1], nrow = r1 - r0;
    // row triangles (the panel's RWGs) and column triangles (those of
    // cells p0..nb-1), each with its position; later[t]: t carries an RWG
    // of a cell after the panel
    std::vector<int32_t> pos(nt, -1), cpos(nt, -1), rows, cols;
    std::vector<char> later(nt, 0);
    for (int b = p0; b < p1; ++b)
      for (int t : ctris[b])
        if (pos[t] < 0) {
          pos[t] = (int32_t)rows.size();
          rows.push_back(t);
        }
    for (int b = p0; b < nb; ++b)
      for (int t : ctris[b]) {
        if (cpos[t] < 0) {
          cpos[t] = (int32_t)cols.size();
          cols.push_back(t);
        }
        if (b >= p1) later[t] = 1;
      }
    std::vector<NearPair> nl, nlt;  // near pairs as they are, and reversed
    for (const NearPair& q : h.near) {
      if (pos[q.p] >= 0 && cpos[q.q] >= 0) nl.push_back({q.p, q.q, pos[q.p], cpos[q.q], q.coplanar, 0});
      if (later[q.p] && pos[q.q] >= 0) nlt.push_back({q.p, q.q, pos[q.q], cpos[q.p], q.coplanar, 0});
    }
    const int64_t nrt = rows.size(), nct = cols.size();
    std::vector<int32_t> redges(h.perm.begin() + r0, h.perm.begin() + r1);
    // entries (panel RWG, later RWG) of the block column that a reversed near
    // pair reaches: the RWGs of its source triangle in the panel against
    // those of its test triangle in the later cells
    std::vector<int32_t> npairs;
    {
      std::vector<int64_t> keys;
      const int64_t nl_later = ne - r1;
      for (const NearPair& q : nlt)
        for (int u = 0; u < 3; ++u) {
          const int64_t ie = h.iperm[h.tri_edge[(size_t)q.q * 3 + u]];
          if (ie < r0 || ie >= r1) continue;
          for (int v = 0; v < 3; ++v) {
            const int64_t jf = h.iperm[h.tri_edge[(size_t)q.p * 3 + v]];
            if (jf >= r1) keys.push_back((ie - r0) * nl_later + (jf - r1));
          }
        }
      std::sort(keys.begin(), keys.end());
      keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
      npairs.reserve(2 * keys.size());
      for (int64_t k : keys) {
        npairs.push_back((int32_t)(k / nl_later));
        npairs.push_back((int32_t)(k % nl_later));
      }
    }
    const size_t ib = 4 * (rows.size() + cols.size() + 2 * pos.size() + redges.size() + npairs.size()) +
                      sizeof(NearPair) * (nl.size() + nlt.size());
    staged.emplace_back(ib);
    std::vector<char>& host = staged.back();
    Scratch idx(ib, s);
    size_t o = 0;
    auto put = [&](const void* src, size_t bytes) {
      if (bytes) std::memcpy(host.data() + o, src, bytes);
      void* d = idx.as<char>() + o;
      o += bytes;
      return d;
    };
    auto* d_rows = (int32_t*)put(rows.data(), 4 * rows.size());
    auto* d_cols = (int32_t*)put(cols.data(), 4 * cols.size());
    auto* d_pos = (int32_t*)put(pos.data(), 4 * pos.size());
    auto* d_cpos = (int32_t*)put(cpos.data(), 4 * cpos.size());
    auto* d_re = (int32_t*)put(redges.data(), 4 * redges.size());
    auto* d_nl = (NearPair*)put(nl.data(), sizeof(NearPair) * nl.size());
    auto* d_nlt = (NearPair*)put(nlt.data(), sizeof(NearPair) * nlt.size());
    auto* d_np = (int32_t*)put(npairs.data(), 4 * npairs.size());
    CBFM_HIP(hipMemcpyAsync(idx.p, host.data(), ib, hipMemcpyHostToDevice, s));
    const int64_t ncol = ne - r0, nlater = ne - r1;
    const int64_t NLc = c->NL - c->off[p0], NLp = c->off[p1] - c->off[p0];
    Scratch local((size_t)27 * nrt * nct * esz, s);
    Scratch Zp((size_t)3 * nrow * ncol * zs, s);
    Scratch W(std::max((size_t)4 * nrow * NLc, (size_t)4 * nlater * NLp) * zs, s);
    fill_local(m, md, fillp, CBFM_LAYOUT_OPS3, d_rows, nrt, d_cols, nct, d_nl, (int64_t)nl.size(), local.p, s);
    // block row: the panel's RWGs against those of cells p0..nb-1
    const int32_t* colEdges = m->perm.as<int32_t>() + r0;
    assemble(m, fillp, local.p, nrt, nct, d_re, nrow, colEdges, ncol, d_pos, d_cpos, Zp.p, nrow * ncol, ncol, s,
             mixed ? 0 : 1);
    {
      std::vector<GemmDesc> d1, d2;
      std::vector<GemmDescX> x1, x2;
      block_gemms(h, c, p0, p1, p0, nb, Zp.p, ncol, false, W.p, mixed, Zr, ldz, d1, d2, x1, x2);
      launch_panel_gemms(precision, d1, d2, x1, x2, s, &keepd, &keepx);
    }
    if (p1 < nb) {
      // block column: the later cells' near pairs against the panel in the
      // reversed slots, the entries they reach re-gathered into the block
      // row's later-cell part, which then holds Z[cells p1..][panel]
      // stored transposed
      fill_near(m, md, fillp, CBFM_LAYOUT_OPS3, d_nlt, (int64_t)nlt.size(), nrt, nct, local.p, s, 1);
      void* Zcol = static_cast<char*>(Zp.p) + (r1 - r0) * zs;
      assemble_pairs(m, fillp, local.p, nrt, nct, d_re, colEdges + (r1 - r0), d_np, (int64_t)npairs.size() / 2, d_pos,
                     d_cpos, Zcol, nrow * ncol, ncol, s, mixed ? 0 : 1);
      std::vector<GemmDesc> d1, d2;
      std::vector<GemmDescX> x1, x2;
      block_gemms(h, c, p1, nb, p0, p1, Zcol, ncol, true, W.p, mixed, Zr, ldz, d1, d2, x1, x2, nrow * ncol);
      launch_panel_gemms(precision, d1, d2, x1, x2, s, &keepd, &keepx);
    }
  }
  CBFM_HIP(hipStreamSynchronize(s));  // the staged host data above is released after this
  return (int)panels.size();
}

// Copy the reduced block of each offset to every cell pair with that
// offset (blockIdx.x = pair a nb + b, blockIdx.y = quadrant: J-M, J-J, M-M,
// M-J).  Zd holds per offset the four L x L row-major quadrants.
__global__ void scatter_offsets_kernel(const double2* __restrict__ Zd, const int32_t* __restrict__ pair_k, int nb,
                                       int64_t L, int64_t NL, double2* __restrict__ Zr, int64_t ldz) {
  const int64_t p = blockIdx.x;
  const int q = blockIdx.y;
  const int64_t a = p / nb, b = p % nb, k = pair_k[p];
  const double2* src = Zd + (k * 4 + q) * L * L;
  const int64_t r0 = (q >= 2 ? NL : 0) + a * L, c0 = (q == 1 || q == 3 ? NL : 0) + b * L;
  for (int64_t e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int64_t i = e / L, j = e % L;
    Zr[(r0 + i) * ldz + c0 + j] = src[e];
  }
}

// Z_r on a mesh of translated copies of cell 0 whose cells share cell 0's
// CBFs (FP64): the block of cells (a, b) is C_0^H Z_ab C_0 and Z_ab depends
// only on the offset of b from a, so each distinct offset is filled
// (regular pairs in one persistent launch, near pairs batched, assembly)
// and projected once, for a representative pair, and copied to the pairs
// that share it.  Offsets are grouped while their scratch fits the budget.
static int project_translated(const cbfm_mesh_s* m, const Media& md, cbfm_cbf_s* c, double2* Zr, int64_t ldz,
                              hipStream_t s, size_t budget) {
  const MeshHost& h = m->h;
  const int nb = h.nblocks;
  const int64_t N0 = h.cell_off[1] - h.cell_off[0], L = c->L[0], NL = c->NL;
  // distinct offsets (coordinates rounded to 1e-7 of the mesh extent) and
  // the first pair of each
  double ext = 0;
  for (int b = 0; b < nb; ++b)
    for (int x = 0; x < 3; ++x) ext = std::max(ext, std::abs(m->shift[(size_t)b * 3 + x]));
  const double unit = std::max(ext, 1e-300) * 1e-7;
  std::map<std::array<int64_t, 3>, int32_t> kof;
  std::vector<std::pair<int, int>> rep;
  std::vector<int32_t> pair_k((size_t)nb * nb);
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      std::array<int64_t, 3> key;
      for (int x = 0; x < 3; ++x)
        key[x] = std::llround((m->shift[(size_t)b * 3 + x] - m->shift[(size_t)a * 3 + x]) / unit);
      auto it = kof.find(key);
      if (it == kof.end()) {
        it = kof.emplace(key, (int32_t)rep.size()).first;
        rep.push_back({a, b});
      }
      pair_k[(size_t)a * nb + b] = it->second;
    }
  const int K = (int)rep.size();
  // each cell's support triangles (ascending) and every triangle's position
  // in its cell's support (one cell per triangle)
  std::vector<std::vector<int32_t>> tris(nb);
  std::vector<int32_t> tpos(h.nt, -1);
  for (int64_t t = 0; t < h.nt; ++t) {
    const int b = m->tcell[t];
    if (b < 0) continue;
    tpos[t] = (int32_t)tris[b].size();
    tris[b].push_back((int32_t)t);
  }
  const int64_t nt0 = (int64_t)tris[0].size();
  for (int b = 0; b < nb; ++b) CBFM_REQUIRE((int64_t)tris[b].size() == nt0, CBFM_E_STATE, "translated cells differ");
  // near pairs of each representative pair, tagged with its offset
  std::vector<int32_t> krep((size_t)nb * nb, -1);
  for (int k = 0; k < K; ++k) krep[(size_t)rep[k].first * nb + rep[k].second] = k;
  std::vector<std::vector<NearPair>> near(K);
  for (const NearPair& q : h.near) {
    const int a = m->tcell[q.p], b = m->tcell[q.q];
    if (a < 0 || b < 0) continue;
    const int k = krep[(size_t)a * nb + b];
    if (k >= 0) near[k].push_back({q.p, q.q, tpos[q.p], tpos[q.q], q.coplanar, k});
  }
  // device tables: supports (cell after cell), positions, near pairs,
  // offset of every pair
  std::vector<int32_t> alltris;
  for (int b = 0; b < nb; ++b) alltris.insert(alltris.end(), tris[b].begin(), tris[b].end());
  std::vector<int64_t> noff(K + 1, 0);
  for (int k = 0; k < K; ++k) noff[k + 1] = noff[k] + (int64_t)near[k].size();
  std::vector<NearPair> allnear;
  allnear.reserve(noff[K]);
  for (int k = 0; k < K; ++k) allnear.insert(allnear.end(), near[k].begin(), near[k].end());
  Scratch dtris(alltris.size() * sizeof(int32_t), s), dpos(tpos.size() * sizeof(int32_t), s),
      dnear(std::max<size_t>(1, allnear.size()) * sizeof(NearPair), s), dpk(pair_k.size() * sizeof(int32_t), s);
  CBFM_HIP(hipMemcpyAsync(dtris.p, alltris.data(), alltris.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  CBFM_HIP(hipMemcpyAsync(dpos.p, tpos.data(), tpos.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (!allnear.empty())
    CBFM_HIP(hipMemcpyAsync(dnear.p, allnear.data(), allnear.size() * sizeof(NearPair), hipMemcpyHostToDevice, s));
  CBFM_HIP(hipMemcpyAsync(dpk.p, pair_k.data(), pair_k.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // reduced blocks of every offset: four L x L quadrants
  Scratch Zd((size_t)K * 4 * L * L * sizeof(double2), s);
  const double2* CM0 = c->CM.as<double2>();
  const double2* CJ0 = c->CJ.as<double2>();
  const size_t loc = (size_t)27 * nt0 * nt0, zb = (size_t)3 * N0 * N0, wb = (size_t)4 * N0 * L;
  const size_t per = (loc + zb + wb) * sizeof(double2);
  const int G = (int)std::max<size_t>(1, std::min<size_t>((size_t)K, budget / per));
  int groups = 0;
  for (int k0 = 0; k0 < K; k0 += G, ++groups) {
    const int k1 = std::min(K, k0 + G), ng = k1 - k0;
    Scratch local((size_t)ng * loc * sizeof(double2), s), Zb((size_t)ng * zb * sizeof(double2), s),
        W((size_t)ng * wb * sizeof(double2), s), outs((size_t)ng * sizeof(NearOut), s);
    std::vector<FillBatchItem> items;
    std::vector<NearOut> hout(ng);
    for (int k = k0; k < k1; ++k) {
      const int a = rep[k].first, b = rep[k].second;
      items.push_back({m, md, CBFM_LAYOUT_OPS3, dtris.as<int32_t>() + (size_t)a * nt0, nt0,
                       dtris.as<int32_t>() + (size_t)b * nt0, nt0, local.as<double2>() + (size_t)(k - k0) * loc});
      hout[k - k0] = {(int64_t)((size_t)(k - k0) * loc), 9 * nt0 * nt0, 3 * nt0};
    }
    CBFM_HIP(hipMemcpyAsync(outs.p, hout.data(), hout.size() * sizeof(NearOut), hipMemcpyHostToDevice, s));
    fill_regular_batch(items, CBFM_FP64, s);  // (synchronises: the near-out table has arrived)
    fill_near_batch(m, md, CBFM_LAYOUT_OPS3, dnear.as<NearPair>() + noff[k0], noff[k1] - noff[k0],
                    outs.as<NearOut>(), k0, local.p, s);
    std::vector<GemmDesc> d1, d2;
    for (int k = k0; k < k1; ++k) {
      const int a = rep[k].first, b = rep[k].second;
      double2* Zk = Zb.as<double2>() + (size_t)(k - k0) * zb;  // K, TE, TH: N0 x N0 each
      assemble(m, CBFM_FP64, local.as<double2>() + (size_t)(k - k0) * loc, nt0, nt0, m->perm.as<int32_t>() + h.cell_off[a],
               N0, m->perm.as<int32_t>() + h.cell_off[b], N0, dpos.as<int32_t>(), dpos.as<int32_t>(), Zk, N0 * N0, N0,
               s, 1);
      double2* Wk = W.as<double2>() + (size_t)(k - k0) * wb;  // K C^M, K C^J, TE C^J, TH C^M: N0 x L each
      const double2* Zop[4] = {Zk, Zk, Zk + N0 * N0, Zk + 2 * N0 * N0};
      const double2* Cop[4] = {CM0, CJ0, CJ0, CM0};
      for (int u = 0; u < 4; ++u) d1.push_back(gemm(Zop[u], N0, OP_N, Cop[u], L, OP_N, Wk + u * N0 * L, L, N0, L, N0));
      // quadrants: J-M = C^J^H K C^M, J-J = -C^J^H TE C^J, M-M = C^M^H TH C^M, M-J = C^M^H K C^J
      double2* Dk = Zd.as<double2>() + (size_t)k * 4 * L * L;
      const double2* Cq[4] = {CJ0, CJ0, CM0, CM0};
      const int wq[4] = {0, 2, 3, 1};
      const double al[4] = {1.0, -1.0, 1.0, 1.0};
      for (int u = 0; u < 4; ++u)
        d2.push_back(gemm(Cq[u], L, OP_C, Wk + wq[u] * N0 * L, L, OP_N, Dk + u * L * L, L, L, L, N0, al[u]));
    }
    zgemm_batched(d1, s);
    zgemm_batched(d2, s);
  }
  CBFM_REQUIRE((int64_t)nb * nb <= 0x7fffffff, CBFM_E_ARG, "too many cell pairs");
  hipLaunchKernelGGL(scatter_offsets_kernel, dim3((unsigned)((int64_t)nb * nb), 4), dim3(256), 0, s, Zd.as<double2>(),
                     dpk.as<int32_t>(), nb, L, NL, Zr, ldz);
  CBFM_HIP(hipGetLastError());
  return groups;
}

// Z_r of several scatterers, each taken as one panel of all its cells: the
// regular fills of all of them in one persistent launch, then per scatterer
// the near pairs and the assembly, then the projection GEMMs of all of them
// in two batched launches.  Consecutive scatterers are grouped while their
// scratch fits the budget; one that does not fit alone goes through the
// panelled single-scatterer path.
struct BatchEntry {
  const cbfm_mesh_s* m;
  Media md;
  cbfm_cbf_s* c;
  double2* Zr;
  int64_t ldz;
};

void project_batch_dev(const std::vector<BatchEntry>& es, int precision, hipStream_t s, size_t budget) {
  const bool mixed = precision == CBFM_MIXED_FP32 || precision == CBFM_MIXED_BF16 || precision == CBFM_MIXED_BF16X3;
  const int fillp = precision == CBFM_FP64 ? CBFM_FP64 : CBFM_FP32;
  const size_t esz = fillp == CBFM_FP64 ? 16 : 8;
  auto full = [&](const BatchEntry& e) {
    const MeshHost& h = e.m->h;
    return panel_bytes(h.nt, h.nt, h.ne, h.ne, 0, e.c->NL, 0, esz, mixed ? sizeof(float2) : sizeof(double2));
  };
  struct Prep {
    std::unique_ptr<Scratch> idx, local, Zp, W;
    int32_t* iota;
    NearPair* near;
  };
  size_t i = 0;
  while (i < es.size()) {
    size_t j = i, bytes = 0;
    while (j < es.size() && (j == i || bytes + full(es[j]) <= budget)) bytes += full(es[j++]);
    if (j == i + 1 && bytes > budget) {
      project_dev(es[i].m, es[i].md, es[i].c, precision, es[i].Zr, es[i].ldz, s, budget);
      i = j;
      continue;
    }
    std::vector<std::unique_ptr<Prep>> preps;
    std::vector<FillBatchItem> items;
    for (size_t k = i; k < j; ++k) {
      const BatchEntry& e = es[k];
      const MeshHost& h = e.m->h;
      auto p = std::make_unique<Prep>();
      std::vector<int32_t> iota(h.nt);
      for (int64_t t = 0; t < h.nt; ++t) iota[t] = (int32_t)t;
      const size_t ib = 4 * iota.size() + sizeof(NearPair) * h.near.size();
      p->idx.reset(new Scratch(ib, s));
      CBFM_HIP(hipMemcpyAsync(p->idx->p, iota.data(), 4 * iota.size(), hipMemcpyHostToDevice, s));
      if (!h.near.empty())
        CBFM_HIP(hipMemcpyAsync(p->idx->as<char>() + 4 * iota.size(), h.near.data(), sizeof(NearPair) * h.near.size(),
                                hipMemcpyHostToDevice, s));
      p->iota = p->idx->as<int32_t>();
      p->near = reinterpret_cast<NearPair*>(p->idx->as<char>() + 4 * iota.size());
      const size_t zsz = mixed ? sizeof(float2) : sizeof(double2);
      p->local.reset(new Scratch((size_t)27 * h.nt * h.nt * esz, s));
      p->Zp.reset(new Scratch((size_t)3 * h.ne * h.ne * zsz, s));
      p->W.reset(new Scratch((size_t)4 * h.ne * e.c->NL * zsz, s));
      items.push_back({e.m, e.md, CBFM_LAYOUT_OPS3, p->iota, h.nt, p->iota, h.nt, p->local->p});
      preps.push_back(std::move(p));
    }
    fill_regular_batch(items, fillp, s);
    std::vector<GemmDesc> d1, d2;
    std::vector<GemmDescX> x1, x2;
    for (size_t k = i; k < j; ++k) {
      const BatchEntry& e = es[k];
      const MeshHost& h = e.m->h;
      Prep& p = *preps[k - i];
      fill_near(e.m, e.md, fillp, CBFM_LAYOUT_OPS3, p.near, (int64_t)h.near.size(), h.nt, h.nt, p.local->p, s);
      assemble(e.m, fillp, p.local->p, h.nt, h.nt, e.m->perm.as<int32_t>(), h.ne, e.m->perm.as<int32_t>(), h.ne,
               p.iota, p.iota, p.Zp->p, h.ne * h.ne, h.ne, s, mixed ? 0 : 1);
      panel_gemms(h, e.c, 0, h.nblocks, p.Zp->p, p.W->p, mixed, e.Zr, e.ldz, d1, d2, x1, x2);
    }
    launch_panel_gemms(precision, d1, d2, x1, x2, s);
    i = j;
  }
}

}  // namespace cbfm

using namespace cbfm;

extern "C" cbfm_status cbfm_project_batch(int32_t count, const cbfm_mesh* meshes, const cbfm_medium* media,
                                          const cbfm_cbf* cbfs, int32_t precision, void* const* Zr, const int64_t* ldz,
                                          void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(count >= 0, CBFM_E_ARG, "negative count");
    if (count == 0) return;
    CBFM_REQUIRE(meshes && media && cbfs && Zr && ldz, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(precision == CBFM_FP64 || precision == CBFM_FP32 || precision == CBFM_MIXED_FP32 ||
                     precision == CBFM_MIXED_BF16 || precision == CBFM_MIXED_BF16X3,
                 CBFM_E_ARG, "unknown precision");
    std::vector<BatchEntry> es;
    for (int32_t k = 0; k < count; ++k) {
      CBFM_REQUIRE(meshes[k] && cbfs[k] && Zr[k], CBFM_E_ARG, "null entry " + std::to_string(k));
      CBFM_REQUIRE(cbfs[k]->mesh == meshes[k], CBFM_E_STATE, "CBF set of entry " + std::to_string(k) + " belongs to another mesh");
      CBFM_REQUIRE(ldz[k] >= 2 * cbfs[k]->NL, CBFM_E_ARG, "ldz < N_CBF in entry " + std::to_string(k));
      CBFM_REQUIRE(meshes[k]->h.nt <= 65535, CBFM_E_ARG, "too many triangles for one assembly launch");
      es.push_back({meshes[k], make_media(&media[k]), cbfs[k], static_cast<double2*>(Zr[k]), ldz[k]});
    }
    size_t fr = 0, tot = 0;
    CBFM_HIP(hipMemGetInfo(&fr, &tot));
    fr += scratch_cached_bytes();  // cached scratch is free for this call's panels
    const size_t budget = std::min<size_t>(fr / 4, (size_t)32 << 30);
    project_batch_dev(es, precision, static_cast<hipStream_t>(stream), budget);
  });
}

extern "C" cbfm_status cbfm_project_ex(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, int32_t precision, void* Zr,
                                       int64_t ldz, int64_t panel_bytes, int32_t* npanels, void* stream) {
  return guarded([&] {
    CBFM_REQUIRE(m && c && Zr, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(c->mesh == m, CBFM_E_STATE, "CBF set belongs to another mesh");
    CBFM_REQUIRE(precision == CBFM_FP64 || precision == CBFM_FP32 || precision == CBFM_MIXED_FP32 ||
                     precision == CBFM_MIXED_BF16 || precision == CBFM_MIXED_BF16X3,
                 CBFM_E_ARG, "unknown precision");
    CBFM_REQUIRE(ldz >= 2 * c->NL, CBFM_E_ARG, "ldz < N_CBF");
    CBFM_REQUIRE(panel_bytes >= 0, CBFM_E_ARG, "negative panel budget");
    const Media md = make_media(med);
    size_t budget = (size_t)panel_bytes;
    if (budget == 0) {
      // scratch budget per panel: a quarter of the free device memory, at most 32 GiB
      size_t fr = 0, tot = 0;
      CBFM_HIP(hipMemGetInfo(&fr, &tot));
      fr += scratch_cached_bytes();  // cached scratch is free for this call's panels
      budget = std::min<size_t>(fr / 4, (size_t)32 << 30);
    }
    int np = 0;
    if (m->translated && c->shared && precision == CBFM_FP64)
      np = project_translated(m, md, c, static_cast<double2*>(Zr), ldz, static_cast<hipStream_t>(stream), budget);
    else
      np = project_dev(m, md, c, precision, static_cast<double2*>(Zr), ldz, static_cast<hipStream_t>(stream), budget);
    if (npanels) *npanels = np;
  });
}

extern "C" cbfm_status cbfm_project(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, int32_t precision, void* Zr,
                                    int64_t ldz, void* stream) {
  return cbfm_project_ex(m, med, c, precision, Zr, ldz, 0, nullptr, stream);
}
