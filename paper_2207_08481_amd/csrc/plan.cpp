// Host planning for the MCS solver: topology, dof numbering, facet colouring,
// multigrid lattice hierarchy and the workspace layout (Sec. 3 of the paper:
// mesh, facets and the discrete spaces; all of the boundary is Dirichlet).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <stdexcept>

#include "kernels_common.h"

namespace mcs {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

std::recursive_mutex& device_api_mutex() {
  static std::recursive_mutex m;
  return m;
}

namespace {

struct Layout {
  size_t bytes = 0;
  std::vector<std::pair<std::string, int64_t>>* names;
  int64_t add(const char* name, size_t nbytes) {
    bytes = (bytes + 255) & ~size_t(255);
    int64_t off = (int64_t)bytes;
    bytes += nbytes;
    names->push_back({name, off});
    return off;
  }
};

int64_t coarse_count(int n) {  // coarse points of n intervals: 0,2,4,.. plus n
  return (n % 2 == 0) ? n / 2 + 1 : (n + 1) / 2 + 1;
}

}  // namespace

// Multigrid levels of all member problems: level l holds one lattice block
// per problem whose hierarchy reaches l, vertices in problem order; the
// block list puts the continuing blocks first.
void build_mg(mcs_problem* pb) {
  int L = 0;
  for (auto& lv : pb->plev) L = std::max(L, (int)lv.size());
  pb->mg.assign(L, MGLevel{});
  std::vector<std::vector<int64_t>> voff(L, std::vector<int64_t>(pb->nprob, -1));
  for (int l = 0; l < L; ++l) {
    int64_t off = 0;
    for (int i = 0; i < pb->nprob; ++i)
      if ((int)pb->plev[i].size() > l) {
        voff[l][i] = off;
        off += pb->plev[i][l].nvert;
      }
    pb->mg[l].nvert = off;
  }
  pb->nc = 0;
  pb->ncinv = 0;
  pb->h_cmap.clear();
  for (int l = 0; l < L; ++l) {
    MGLevel& M = pb->mg[l];
    std::vector<MGBlock> cont, coarse;
    for (int i = 0; i < pb->nprob; ++i) {
      const auto& lv = pb->plev[i];
      if ((int)lv.size() <= l) continue;
      MGBlock B{};
      B.prob = i;
      B.ffm = pb->pffm[i];
      for (int a = 0; a < 3; ++a) B.n[a] = lv[l].n[a];
      B.nvert = lv[l].nvert;
      B.voff = voff[l][i];
      B.coarsest = (l + 1 == (int)lv.size()) ? 1 : 0;
      if (!B.coarsest) {
        for (int a = 0; a < 3; ++a) B.nc3[a] = lv[l + 1].n[a];
        B.nvert_c = lv[l + 1].nvert;
        B.cvoff = voff[l + 1][i];
        cont.push_back(B);
      } else {
        B.nc = lv[l].nfree;
        B.cmap_off = pb->nc;
        B.cinv_off = pb->ncinv;
        pb->nc += B.nc;
        pb->ncinv += B.nc * B.nc;
        pb->h_cmap.insert(pb->h_cmap.end(), pb->pcmap[i].begin(), pb->pcmap[i].end());
        coarse.push_back(B);
      }
    }
    M.ncont = (int)cont.size();
    M.blocks = cont;
    M.blocks.insert(M.blocks.end(), coarse.begin(), coarse.end());
    M.maxv = M.maxvc = M.maxnc = 0;
    for (auto& B : cont) {
      M.maxv = std::max(M.maxv, B.nvert);
      M.maxvc = std::max(M.maxvc, B.nvert_c);
    }
    for (auto& B : coarse) M.maxnc = std::max(M.maxnc, B.nc);
  }
}

// Builds everything the device needs except the numerical tables.
int plan_problem(const mcs_mesh* mesh, const mcs_options* opt, mcs_problem* pb) {
  const int d = mesh->dim;
  if (d != 2 && d != 3) {
    set_error("dim must be 2 or 3 (got %d)", d);
    return MCS_ERR_ARG;
  }
  const int k = opt->order;
  if (k < 1 || k > 5) {
    set_error("order k must be in 1..5 (got %d)", k);
    return k < 1 ? MCS_ERR_ARG : MCS_ERR_UNSUPPORTED;
  }
  if (k == 1 && d != 3) {
    set_error("the lowest order k = 1 is the three-dimensional method (H(div) omega, Sec. 7)");
    return MCS_ERR_ARG;
  }
  if (mesh->n_vertices <= d || mesh->n_elements <= 0 || !mesh->vertices_host || !mesh->elements_host) {
    set_error("empty mesh");
    return MCS_ERR_ARG;
  }
  for (int a = 0; a < d; ++a)
    if (mesh->lattice[a] < 2) {
      set_error("vertices do not form the declared lattice");
      return MCS_ERR_MESH;
    }
  int ffm = 0;
  for (int a = 0; a < 2 * d; ++a) {
    if (mesh->face_bc[a] != 0 && mesh->face_bc[a] != 1) {
      set_error("face_bc[%d] must be 0 (Dirichlet) or 1 (outlet)", a);
      return MCS_ERR_ARG;
    }
    if (mesh->face_bc[a] == 1) ffm |= 1 << a;
  }
  pb->pffm.assign(1, ffm);
  pb->d = d;
  pb->opt = *opt;
  if (pb->opt.smoothing_steps <= 0) pb->opt.smoothing_steps = 2;
  if (pb->opt.max_it <= 0) pb->opt.max_it = 1000;
  if (!(pb->opt.tol > 0)) pb->opt.tol = 1e-10;
  if (!(pb->opt.inner_tol > 0)) pb->opt.inner_tol = 1e-5;
  if (pb->opt.max_outer <= 0) pb->opt.max_outer = 10;
  if (pb->opt.coarse_max <= 0) pb->opt.coarse_max = 512;
  if (pb->opt.precision != 0 && pb->opt.precision != 1) {
    set_error("precision must be 0 or 1");
    return MCS_ERR_ARG;
  }
  if (pb->opt.smoother < 0 || pb->opt.smoother > 3) {
    set_error("smoother must be 0 (multiplicative, block Gauss-Seidel), 1 (additive, facet block Jacobi), 2 "
              "(full system, overlapping block Gauss-Seidel) or 3 (multiplicative, facet block l1-Jacobi)");
    return MCS_ERR_ARG;
  }
  pb->sz = make_sizes(d, k);
  if (k == 1 && pb->opt.smoother == 2) {
    set_error("k = 1 has no velocity bubbles: the full-system variant is the condensed one (smoother 0)");
    return MCS_ERR_UNSUPPORTED;
  }
  if (pb->opt.smoother == 2) {
    const int nbk = pb->sz.nfb + 2 * pb->sz.nb;
    if (pb->opt.precision != 0 || nbk > 64) {
      set_error("the full-system variant needs precision 0 and blocks of at most 64 dofs (n_fb + 2 n_b = %d)", nbk);
      return MCS_ERR_UNSUPPORTED;
    }
  }
  const Sizes& s = pb->sz;
  const int nv = d + 1;
  const int64_t ne = mesh->n_elements, nvert = mesh->n_vertices;
  pb->ne = ne;
  pb->nvert = nvert;
  pb->h_coords.assign(mesh->vertices_host, mesh->vertices_host + nvert * d);
  for (int64_t i = 0; i < nvert * d; ++i)
    if (!std::isfinite(pb->h_coords[i])) {
      set_error("non-finite vertex coordinate");
      return MCS_ERR_ARG;
    }

  // ---- sorted element vertices and permutation ranks
  pb->h_elem_verts.resize(ne * nv);
  pb->h_elem_perm.resize(ne);
  for (int64_t e = 0; e < ne; ++e) {
    std::array<int, 4> idx{0, 1, 2, 3};
    const int32_t* ev = mesh->elements_host + e * nv;
    for (int j = 0; j < nv; ++j)
      if (ev[j] < 0 || ev[j] >= nvert) {
        set_error("element %lld references vertex %d out of range", (long long)e, ev[j]);
        return MCS_ERR_MESH;
      }
    std::sort(idx.begin(), idx.begin() + nv, [&](int a, int b) { return ev[a] < ev[b]; });
    for (int j = 0; j + 1 < nv; ++j)
      if (ev[idx[j]] == ev[idx[j + 1]]) {
        set_error("element %lld has a repeated vertex", (long long)e);
        return MCS_ERR_MESH;
      }
    for (int j = 0; j < nv; ++j) pb->h_elem_verts[e * nv + j] = ev[idx[j]];
    pb->h_elem_perm[e] = perm_index(idx.data(), nv);
    // degenerate element check
    double J[3][3] = {};
    const double* X0 = &pb->h_coords[(size_t)ev[idx[0]] * d];
    for (int c = 0; c < d; ++c) {
      const double* Xc = &pb->h_coords[(size_t)ev[idx[c + 1]] * d];
      for (int r = 0; r < d; ++r) J[r][c] = Xc[r] - X0[r];
    }
    double det = (d == 2) ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                          : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double h = 0;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) h = std::max(h, std::fabs(J[r][c]));
    if (!(std::fabs(det) > 1e-12 * std::pow(h, d))) {
      set_error("element %lld is degenerate", (long long)e);
      return MCS_ERR_MESH;
    }
  }

  // ---- facets in canonical order
  struct FI {
    std::array<int32_t, 3> v;
    int32_t e;
    int8_t slot;
  };
  std::vector<FI> fl;
  fl.reserve(ne * nv);
  for (int64_t e = 0; e < ne; ++e)
    for (int i = 0; i < nv; ++i) {
      FI f{{-1, -1, -1}, (int32_t)e, (int8_t)i};
      int c = 0;
      for (int j = 0; j < nv; ++j)
        if (j != i) f.v[c++] = pb->h_elem_verts[e * nv + j];
      fl.push_back(f);
    }
  std::sort(fl.begin(), fl.end(), [](const FI& a, const FI& b) {
    if (a.v != b.v) return a.v < b.v;
    return a.e < b.e;
  });
  pb->h_elem_ff.assign(ne * nv, -1);
  std::vector<std::array<int32_t, 3>> free_fv;
  std::vector<uint8_t> vbound(nvert, 0);
  for (size_t i = 0; i < fl.size();) {
    size_t j = i;
    while (j < fl.size() && fl[j].v == fl[i].v) ++j;
    if (j - i > 2) {
      set_error("a facet is shared by more than two elements");
      return MCS_ERR_MESH;
    }
    // a boundary facet lies on one face of the lattice box: an outlet face
    // keeps it as a free facet with one neighbour
    bool outlet = false;
    if (j - i == 1)
      for (int a = 0; a < d; ++a)
        for (int side = 0; side < 2; ++side) {
          if (!((ffm >> (2 * a + side)) & 1)) continue;
          const int target = side ? mesh->lattice[a] - 1 : 0;
          bool all = true;
          for (int c = 0; c < d; ++c) {
            const int64_t v = fl[i].v[c];
            const int64_t ca = a == 0 ? v % mesh->lattice[0]
                             : a == 1 ? (v / mesh->lattice[0]) % mesh->lattice[1]
                                      : v / ((int64_t)mesh->lattice[0] * mesh->lattice[1]);
            if (ca != target) all = false;
          }
          if (all) outlet = true;
        }
    if (j - i == 1 && !outlet) {
      for (int c = 0; c < d; ++c) vbound[fl[i].v[c]] = 1;
      pb->h_blk_el.insert(pb->h_blk_el.end(), {fl[i].e, -1});
      pb->h_blk_slot.insert(pb->h_blk_slot.end(), {(int32_t)fl[i].slot, -1});
      pb->h_blk_g.push_back(-1);
    } else if (j - i == 1) {
      pb->h_blk_el.insert(pb->h_blk_el.end(), {fl[i].e, -1});
      pb->h_blk_slot.insert(pb->h_blk_slot.end(), {(int32_t)fl[i].slot, -1});
      pb->h_blk_g.push_back((int32_t)free_fv.size());
      const int32_t g = (int32_t)free_fv.size();
      free_fv.push_back(fl[i].v);
      pb->h_facet_el.push_back(fl[i].e);
      pb->h_facet_el.push_back(-1);
      pb->h_facet_slot.push_back(fl[i].slot);
      pb->h_facet_slot.push_back(-1);
      pb->h_facet_out.push_back(1);
      pb->h_elem_ff[fl[i].e * nv + fl[i].slot] = g;
      pb->has_outlet = true;
    } else {
      pb->h_blk_el.insert(pb->h_blk_el.end(), {fl[i].e, fl[i + 1].e});
      pb->h_blk_slot.insert(pb->h_blk_slot.end(), {(int32_t)fl[i].slot, (int32_t)fl[i + 1].slot});
      pb->h_blk_g.push_back((int32_t)free_fv.size());
      int32_t g = (int32_t)free_fv.size();
      free_fv.push_back(fl[i].v);
      pb->h_facet_el.push_back(fl[i].e);
      pb->h_facet_el.push_back(fl[i + 1].e);
      pb->h_facet_slot.push_back(fl[i].slot);
      pb->h_facet_slot.push_back(fl[i + 1].slot);
      pb->h_facet_out.push_back(0);
      pb->h_elem_ff[fl[i].e * nv + fl[i].slot] = g;
      pb->h_elem_ff[fl[i + 1].e * nv + fl[i + 1].slot] = g;
    }
    i = j;
  }
  const int64_t nff = (int64_t)free_fv.size();
  pb->nff = nff;

  // ---- greedy colouring in canonical order
  pb->h_colour.assign(nff, -1);
  int ncol = 0;
  for (int64_t g = 0; g < nff; ++g) {
    uint32_t used = 0;
    for (int side = 0; side < 2; ++side) {
      int64_t e = pb->h_facet_el[2 * g + side];
      if (e < 0) continue;
      for (int i = 0; i < nv; ++i) {
        int32_t g2 = pb->h_elem_ff[e * nv + i];
        if (g2 >= 0 && g2 != g && pb->h_colour[g2] >= 0) used |= 1u << pb->h_colour[g2];
      }
    }
    int c = 0;
    while (used & (1u << c)) ++c;
    pb->h_colour[g] = c;
    ncol = std::max(ncol, c + 1);
  }
  pb->ncol = ncol;
  pb->colour_off.assign(ncol + 1, 0);
  for (int64_t g = 0; g < nff; ++g) pb->colour_off[pb->h_colour[g] + 1]++;
  for (int c = 0; c < ncol; ++c) pb->colour_off[c + 1] += pb->colour_off[c];
  pb->h_colour_facets.resize(nff);
  {
    std::vector<int32_t> pos(pb->colour_off.begin(), pb->colour_off.end() - 1);
    for (int64_t g = 0; g < nff; ++g) pb->h_colour_facets[pos[pb->h_colour[g]]++] = (int32_t)g;
  }

  // ---- blocks of the full-system variant: greedy colouring of all facets in
  // canonical order, the smallest colour not used by a facet of a neighbour
  pb->nblk = (int64_t)pb->h_blk_g.size();
  {
    const int64_t nblk = pb->nblk;
    std::vector<int32_t> elem_blk(ne * nv, -1);
    for (int64_t b = 0; b < nblk; ++b)
      for (int side = 0; side < 2; ++side)
        if (pb->h_blk_el[2 * b + side] >= 0) elem_blk[pb->h_blk_el[2 * b + side] * nv + pb->h_blk_slot[2 * b + side]] = (int32_t)b;
    pb->h_blk_colour.assign(nblk, -1);
    int nc = 0;
    for (int64_t b = 0; b < nblk; ++b) {
      uint32_t used = 0;
      for (int side = 0; side < 2; ++side) {
        const int64_t e = pb->h_blk_el[2 * b + side];
        if (e < 0) continue;
        for (int i = 0; i < nv; ++i) {
          const int32_t b2 = elem_blk[e * nv + i];
          if (b2 != b && pb->h_blk_colour[b2] >= 0) used |= 1u << pb->h_blk_colour[b2];
        }
      }
      int c = 0;
      while (used & (1u << c)) ++c;
      pb->h_blk_colour[b] = c;
      nc = std::max(nc, c + 1);
    }
    pb->ncol_full = nc;
    pb->colour_off_full.assign(nc + 1, 0);
    for (int64_t b = 0; b < nblk; ++b) pb->colour_off_full[pb->h_blk_colour[b] + 1]++;
    for (int c = 0; c < nc; ++c) pb->colour_off_full[c + 1] += pb->colour_off_full[c];
    pb->h_colour_blocks.resize(nblk);
    std::vector<int32_t> pos(pb->colour_off_full.begin(), pb->colour_off_full.end() - 1);
    for (int64_t b = 0; b < nblk; ++b) pb->h_colour_blocks[pos[pb->h_blk_colour[b]]++] = (int32_t)b;
    // algorithmic bytes of a colour phase: per block its inverse (m^2), the
    // columns of A_T of both neighbours for its dofs in that element
    // ((n_F-dofs + n_b) x n_A each), the gathered products and the updated x
    const Sizes& z = pb->sz;
    pb->full_colour_bytes.assign(nc, 0.0);
    for (int64_t b = 0; b < nblk; ++b) {
      const int nf = pb->h_blk_g[b] >= 0 ? z.nfb : 0;
      const int nside = pb->h_blk_el[2 * b + 1] >= 0 ? 2 : 1;
      const int m = nf + nside * z.nb;
      const double words = (double)m * m + (double)nside * (nf + z.nb) * z.nA + 2.0 * nside * (nf + z.nb) + 3.0 * m +
                           2.0 * nside * z.nA;
      pb->full_colour_bytes[pb->h_blk_colour[b]] += 8.0 * words + 4.0 * 5;
    }
  }

  // ---- free vertices (P1 auxiliary space)
  std::vector<int32_t> vfree(nvert, -1);
  int64_t nfv = 0;
  for (int64_t v = 0; v < nvert; ++v)
    if (!vbound[v]) vfree[v] = (int32_t)nfv++;
  pb->nfv = nfv;
  pb->h_vfree_of_lat = vfree;
  pb->h_free_to_lat.assign(nfv, 0);
  for (int64_t v = 0; v < nvert; ++v)
    if (vfree[v] >= 0) pb->h_free_to_lat[vfree[v]] = (int32_t)v;
  pb->h_facet_vfree.resize(nff * d);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> inc(nfv);
  for (int64_t g = 0; g < nff; ++g)
    for (int c = 0; c < d; ++c) {
      int32_t fv = vfree[free_fv[g][c]];
      pb->h_facet_vfree[g * d + c] = fv;
      if (fv >= 0) inc[fv].push_back({(int32_t)g, c});
    }
  pb->h_vinc_off.assign(nfv + 1, 0);
  for (int64_t v = 0; v < nfv; ++v) pb->h_vinc_off[v + 1] = pb->h_vinc_off[v] + (int32_t)inc[v].size();
  pb->h_vinc.clear();
  for (int64_t v = 0; v < nfv; ++v)
    for (auto& pr : inc[v]) {
      pb->h_vinc.push_back(pr.first);
      pb->h_vinc.push_back(pr.second);
    }
  // lattice vertex -> elements
  {
    std::vector<int32_t> cnt(nvert + 1, 0);
    for (int64_t e = 0; e < ne; ++e)
      for (int j = 0; j < nv; ++j) cnt[pb->h_elem_verts[e * nv + j] + 1]++;
    for (int64_t v = 0; v < nvert; ++v) cnt[v + 1] += cnt[v];
    pb->h_vert_elem_off = cnt;
    pb->h_vert_elem.assign(cnt[nvert], 0);
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
      for (int j = 0; j < nv; ++j) pb->h_vert_elem[pos[pb->h_elem_verts[e * nv + j]]++] = (int32_t)e;
  }

  // ---- lattice and multigrid plan
  int64_t lat_n = 1;
  for (int a = 0; a < 3; ++a) pb->lattice[a] = a < d ? mesh->lattice[a] : 1;
  for (int a = 0; a < d; ++a) lat_n *= pb->lattice[a];
  if (lat_n != nvert || *std::min_element(pb->lattice, pb->lattice + d) < 2) {
    set_error("vertices do not form the declared lattice");
    return MCS_ERR_MESH;
  }
  // every element must lie in one lattice cell and interior lattice vertices must be free
  for (int64_t e = 0; e < ne; ++e) {
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int j = 0; j < nv; ++j) {
      int64_t v = pb->h_elem_verts[e * nv + j];
      int c[3] = {int(v % pb->lattice[0]), int((v / pb->lattice[0]) % pb->lattice[1]),
                  int(v / ((int64_t)pb->lattice[0] * pb->lattice[1]))};
      for (int a = 0; a < d; ++a) {
        lo[a] = std::min(lo[a], c[a]);
        hi[a] = std::max(hi[a], c[a]);
      }
    }
    for (int a = 0; a < d; ++a)
      if (hi[a] - lo[a] > 1) {
        set_error("element %lld spans more than one lattice cell", (long long)e);
        return MCS_ERR_MESH;
      }
  }
  for (int64_t v = 0; v < nvert; ++v) {
    int c[3] = {int(v % pb->lattice[0]), int((v / pb->lattice[0]) % pb->lattice[1]),
                int(v / ((int64_t)pb->lattice[0] * pb->lattice[1]))};
    const int nint[3] = {pb->lattice[0] - 1, pb->lattice[1] - 1, pb->lattice[2] - 1};
    if (lat_free(c, nint, d, ffm) != (vfree[v] >= 0)) {
      set_error("boundary of the mesh does not match the lattice boundary");
      return MCS_ERR_MESH;
    }
  }
  pb->plev.assign(1, {});
  pb->pcmap.assign(1, {});
  {
    int n[3] = {pb->lattice[0] - 1, pb->lattice[1] - 1, d == 3 ? pb->lattice[2] - 1 : 0};
    while (true) {
      LatLevel L{};
      L.n[0] = n[0];
      L.n[1] = n[1];
      L.n[2] = n[2];
      L.nvert = (int64_t)(n[0] + 1) * (n[1] + 1) * (d == 3 ? n[2] + 1 : 1);
      // free vertices per axis: the interior ones plus outlet ends
      int64_t nf = d;
      for (int a = 0; a < d; ++a) nf *= n[a] - 1 + ((ffm >> (2 * a)) & 1) + ((ffm >> (2 * a + 1)) & 1);
      L.nfree = nf;
      pb->plev[0].push_back(L);
      int nmin = std::min(n[0], n[1]);
      if (d == 3) nmin = std::min(nmin, n[2]);
      if (L.nfree <= pb->opt.coarse_max || nmin <= 2) break;
      for (int a = 0; a < d; ++a) n[a] = (int)coarse_count(n[a]) - 1;
    }
    const LatLevel& C = pb->plev[0].back();
    int N0 = C.n[0] + 1, N1 = C.n[1] + 1;
    for (int64_t v = 0; v < C.nvert; ++v) {
      int c[3] = {int(v % N0), int((v / N0) % N1), int(v / ((int64_t)N0 * N1))};
      if (lat_free(c, C.n, d, ffm))
        for (int cc = 0; cc < d; ++cc) pb->pcmap[0].push_back((int32_t)(v * d + cc));
    }
  }
  pb->nprob = 1;
  pb->pe0 = {0, ne};
  pb->pf0 = {0, nff};
  pb->pv0 = {0, nvert};
  pb->pfv0 = {0, nfv};
  build_mg(pb);

  // ---- global layout
  pb->off_f = ne * s.nb;
  pb->off_p = pb->off_f + nff * s.nfb;
  pb->ndof = pb->off_p + ne * s.np;
  pb->np1 = nfv * d;
  return MCS_OK;
}

// Union of planned problems with the same dimension, order and options: the
// host arrays are the members' arrays concatenated in member order, with
// element, facet, vertex and free-vertex indices shifted by the member's
// offsets.  Facet colours are kept (a colour class of the union is the union
// of the members' classes), so every member sees exactly its own topology.
int plan_union(const std::vector<const mcs_problem*>& parts, mcs_problem* u) {
  if (parts.empty()) {
    set_error("empty union");
    return MCS_ERR_ARG;
  }
  const mcs_problem* p0 = parts[0];
  for (auto* q : parts)
    if (q->d != p0->d || q->sz.k != p0->sz.k) {
      set_error("union members must share dimension and order");
      return MCS_ERR_ARG;
    }
  const int d = p0->d, nv = d + 1;
  u->sz = p0->sz;
  u->opt = p0->opt;
  u->d = d;
  for (int a = 0; a < 3; ++a) u->lattice[a] = 0;
  u->nprob = (int)parts.size();
  u->pffm.clear();
  for (auto* q : parts) u->pffm.push_back(q->pffm[0]);
  u->pe0.assign(1, 0);
  u->pf0.assign(1, 0);
  u->pv0.assign(1, 0);
  u->pfv0.assign(1, 0);
  u->plev.clear();
  u->pcmap.clear();
  u->ncol = 0;
  for (auto* q : parts) {
    u->pe0.push_back(u->pe0.back() + q->ne);
    u->pf0.push_back(u->pf0.back() + q->nff);
    u->pv0.push_back(u->pv0.back() + q->nvert);
    u->pfv0.push_back(u->pfv0.back() + q->nfv);
    u->plev.push_back(q->plev[0]);
    u->pcmap.push_back(q->pcmap[0]);
    u->ncol = std::max(u->ncol, q->ncol);
  }
  const int np = u->nprob;
  u->ne = u->pe0[np];
  u->nff = u->pf0[np];
  u->nvert = u->pv0[np];
  u->nfv = u->pfv0[np];
  auto cat = [&](auto member, auto& out, auto shift) {
    out.clear();
    for (int i = 0; i < np; ++i) {
      const auto& src = parts[i]->*member;
      for (auto v : src) out.push_back(shift(i, v));
    }
  };
  auto keep = [](int, int32_t v) { return v; };
  cat(&mcs_problem::h_elem_ff, u->h_elem_ff, [&](int i, int32_t g) { return g >= 0 ? (int32_t)(g + u->pf0[i]) : g; });
  cat(&mcs_problem::h_elem_verts, u->h_elem_verts, [&](int i, int32_t v) { return (int32_t)(v + u->pv0[i]); });
  cat(&mcs_problem::h_elem_perm, u->h_elem_perm, keep);
  cat(&mcs_problem::h_facet_el, u->h_facet_el, [&](int i, int32_t e) { return (int32_t)(e + u->pe0[i]); });
  cat(&mcs_problem::h_facet_slot, u->h_facet_slot, keep);
  cat(&mcs_problem::h_colour, u->h_colour, keep);
  cat(&mcs_problem::h_facet_out, u->h_facet_out, keep);
  cat(&mcs_problem::h_facet_vfree, u->h_facet_vfree, [&](int i, int32_t v) { return v >= 0 ? (int32_t)(v + u->pfv0[i]) : v; });
  cat(&mcs_problem::h_vfree_of_lat, u->h_vfree_of_lat, [&](int i, int32_t v) { return v >= 0 ? (int32_t)(v + u->pfv0[i]) : v; });
  cat(&mcs_problem::h_free_to_lat, u->h_free_to_lat, [&](int i, int32_t v) { return (int32_t)(v + u->pv0[i]); });
  u->h_coords.clear();
  for (auto* q : parts) u->h_coords.insert(u->h_coords.end(), q->h_coords.begin(), q->h_coords.end());
  // CSR arrays: free vertex -> (facet, slot) and vertex -> elements
  u->h_vinc_off.assign(1, 0);
  u->h_vinc.clear();
  u->h_vert_elem_off.assign(1, 0);
  u->h_vert_elem.clear();
  for (int i = 0; i < np; ++i) {
    const mcs_problem* q = parts[i];
    const int32_t b0 = u->h_vinc_off.back();
    for (int64_t v = 0; v < q->nfv; ++v) u->h_vinc_off.push_back(b0 + q->h_vinc_off[v + 1]);
    for (size_t t = 0; t < q->h_vinc.size(); t += 2) {
      u->h_vinc.push_back((int32_t)(q->h_vinc[t] + u->pf0[i]));
      u->h_vinc.push_back(q->h_vinc[t + 1]);
    }
    const int32_t e0 = u->h_vert_elem_off.back();
    for (int64_t v = 0; v < q->nvert; ++v) u->h_vert_elem_off.push_back(e0 + q->h_vert_elem_off[v + 1]);
    for (auto e : q->h_vert_elem) u->h_vert_elem.push_back((int32_t)(e + u->pe0[i]));
  }
  // colour classes
  const int64_t nff = u->nff;
  u->colour_off.assign(u->ncol + 1, 0);
  for (int64_t g = 0; g < nff; ++g) u->colour_off[u->h_colour[g] + 1]++;
  for (int c = 0; c < u->ncol; ++c) u->colour_off[c + 1] += u->colour_off[c];
  u->h_colour_facets.resize(nff);
  {
    std::vector<int32_t> pos(u->colour_off.begin(), u->colour_off.end() - 1);
    for (int64_t g = 0; g < nff; ++g) u->h_colour_facets[pos[u->h_colour[g]]++] = (int32_t)g;
  }
  build_mg(u);
  const Sizes& s = u->sz;
  u->off_f = u->ne * s.nb;
  u->off_p = u->off_f + nff * s.nfb;
  u->ndof = u->off_p + u->ne * s.np;
  u->np1 = u->nfv * d;
  (void)nv;
  return MCS_OK;
}

int layout_workspace(mcs_problem* pb) {
  const Sizes& s = pb->sz;
  const int d = pb->d, nv = d + 1;
  const int64_t ne = pb->ne, nff = pb->nff;
  Layout L;
  pb->offsets.clear();
  L.names = &pb->offsets;
  auto I = [](int64_t n) { return size_t(n) * 4; };
  auto Dd = [](int64_t n) { return size_t(n) * 8; };
  auto Ff = [](int64_t n) { return size_t(n) * 4; };
  L.add("elem_ff", I(ne * nv));
  L.add("elem_verts", I(ne * nv));
  L.add("elem_perm", I(ne));
  L.add("facet_el", I(nff * 2));
  L.add("facet_slot", I(nff * 2));
  L.add("colour_desc", I(nff * 4));
  L.add("facet_out", I(nff));
  L.add("xD", Dd(ne * s.nd));
  L.add("facet_vfree", I(nff * d));
  L.add("vinc_off", I(pb->nfv + 1));
  L.add("vinc", I(pb->h_vinc.size()));
  L.add("vert_elem_off", I(pb->nvert + 1));
  L.add("vert_elem", I(pb->h_vert_elem.size()));
  L.add("coords", Dd(pb->nvert * d));
  L.add("vfree_of_lat", I(pb->nvert));
  L.add("free_to_lat", I(pb->nfv + 1));
  const RefTables& r = pb->ref;
  L.add("rV", Dd(r.V.size()));
  L.add("rBf", Dd(r.Bf.size()));
  L.add("rU", Dd(r.U.size()));
  L.add("rL", Dd(r.L.size()));
  L.add("rLam", Dd(r.Lam.size()));
  L.add("rD", Dd(r.D.size()));
  L.add("rBp", Dd(r.Bp.size()));
  L.add("rMp", Dd(r.Mp.size()));
  L.add("rMpinv", Dd(r.Mpinv.size()));
  L.add("rRf", Dd(r.Rf.size()));
  L.add("rcn", Dd(r.cn.size()));
  L.add("rct", Dd(r.ct.size()));
  L.add("rpconst", Dd(r.pconst.size()));
  L.add("rpmom", Dd(r.pmom.size()));
  L.add("rphi", Dd(r.phi.size()));
  L.add("rpidx", Dd(r.pidx.size()));
  L.add("rpsi", Dd(r.psi.size()));
  L.add("rpsib", Dd(r.psib.size()));
  L.add("rlatmap", I(r.latmap.size()));
  L.add("nu", Dd(ne));
  L.add("detJ", Dd(ne));
  // Precision 1 needs FP64 operators only for the outer residual: A^d, H,
  // A_oo as FP32 hi + lo pairs (hi doubles as the FP32 operator), no FP64
  // preconditioner data.
  pb->lean = pb->opt.precision == 1;
  if (!pb->lean) {
    L.add("Ad", Dd(ne * s.nd * s.nd));
    L.add("H", Dd(ne * s.nb * s.nd));
    L.add("Aoo", Dd(ne * s.nb * s.nb));
    L.add("Aooinv", Dd(ne * s.nb * s.nb));
  }
  L.add("Ad32", Ff(ne * s.nd * s.nd));
  L.add("H32", Ff(ne * s.nb * s.nd));
  L.add("Aoo32", Ff(ne * s.nb * s.nb));
  L.add("Aooinv32", Ff(ne * s.nb * s.nb));
  if (pb->lean) {
    L.add("Adl", Ff(ne * s.nd * s.nd));
    L.add("Hl", Ff(ne * s.nb * s.nd));
    L.add("Aool", Ff(ne * s.nb * s.nb));
  } else {
    L.add("Dinv", Dd(nff * s.nfb * s.nfb));
    L.add("DinvP", Dd(nff * s.nfb * (s.nfb + 1) / 2));
  }
  L.add("EF", Dd(nff * s.nfb * d * d));
  L.add("Dinv32", Ff(nff * s.nfb * s.nfb));
  L.add("DinvP32", Ff(nff * s.nfb * (s.nfb + 1) / 2));
  L.add("EF32", Ff(nff * s.nfb * d * d));
  if (!pb->lean) L.add("W", Dd(ne * (d + 1) * d * s.nd));
  L.add("W32", Ff(ne * (d + 1) * d * s.nd));
  const int st = d == 3 ? 27 : 9;
  for (size_t l = 0; l < pb->mg.size(); ++l) {
    MGLevel& M = pb->mg[l];
    char nm[32];
    snprintf(nm, sizeof nm, "mgA%zu", l);
    M.off_A = L.add(nm, Dd(M.nvert * st * d * d) + Ff(M.nvert * st * d * d));
    snprintf(nm, sizeof nm, "mgDinv%zu", l);
    M.off_Dinv = L.add(nm, Dd(M.nvert * d * d) + Ff(M.nvert * d * d));
    snprintf(nm, sizeof nm, "mgx%zu", l);
    M.off_x = L.add(nm, Dd(M.nvert * d));
    snprintf(nm, sizeof nm, "mgb%zu", l);
    M.off_b = L.add(nm, Dd(M.nvert * d));
    snprintf(nm, sizeof nm, "mgr%zu", l);
    M.off_r = L.add(nm, Dd(M.nvert * d));
    snprintf(nm, sizeof nm, "mgblk%zu", l);
    M.off_blk = L.add(nm, sizeof(MGBlockDev) * M.blocks.size());
  }
  L.add("Cinv", Dd(pb->ncinv));
  L.add("cmap", I(pb->nc));
  pb->n_slots = std::min<int64_t>(ne, 2048);
  pb->slot_doubles = (int64_t)s.nA * s.nsig + (int64_t)s.nlam * s.nsig * 2 + (int64_t)s.nA * s.nlam +
                     (int64_t)s.nA * s.nA + (int64_t)s.nlam * s.nlam + (int64_t)s.nb * s.nb * 2 + 64;
  L.add("cscratch", Dd(pb->n_slots * pb->slot_doubles));
  if (pb->lean) L.add("adtmp", Dd(pb->n_slots * s.nd * s.nd));
  L.add("escr", Dd(ne * s.nd));
  L.add("escr2", Dd(ne * s.nd));
  L.add("fscr", Dd(nff * d * d));
  pb->nred = 4096;
  L.add("red", Dd(pb->nred));
  L.add("scal", Dd(256));
  L.add("wcount", 2 * 256 * 16 * 8);
  if (pb->opt.smoother == 2) {
    const int64_t nbk = s.nfb + 2 * s.nb, nvd = (int64_t)(d + 1) * d;
    L.add("blk_el", I(pb->nblk * 2));
    L.add("blk_slot", I(pb->nblk * 2));
    L.add("blk_g", I(pb->nblk));
    L.add("colour_blocks", I(pb->nblk));
    L.add("Afull", Dd(ne * s.nA * s.nA));
    L.add("Binv", Dd(pb->nblk * nbk * nbk));
    L.add("Wfull", Dd(ne * nvd * s.nA));
    L.add("Eo", Dd(ne * s.nb * nvd));
    L.add("Eoref", Dd(nvd * s.nb));
    L.add("yfull", Dd(ne * s.nA));
    L.add("eto", Dd(ne * nvd));
  }
  // FP64 slots: the MINRES and K-hat vectors, then b, r, x, K x of the
  // refinement (the only ones the lean layout keeps)
  pb->vbase64 = pb->lean ? 15 : 0;
  pb->nvec64 = pb->lean ? 4 : 24;
  pb->nvec32 = 20;
  L.add("vec", Dd(pb->ndof * pb->nvec64));
  L.add("vec32", Ff(pb->ndof * pb->nvec32));
  L.add("p1", Dd(pb->np1 * 4 + 16));
  L.add("p132", Ff(pb->np1 * 4 + 16));
  pb->ws_bytes = (L.bytes + 4095) & ~size_t(4095);
  return MCS_OK;
}

int64_t offset_of(const mcs_problem* pb, const char* name) {
  for (auto& pr : pb->offsets)
    if (pr.first == name) return pr.second;
  return -1;
}

}  // namespace mcs
