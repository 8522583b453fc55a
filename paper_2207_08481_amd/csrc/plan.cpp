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

#include "mcs_internal.h"

namespace mcs {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

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

// Builds everything the device needs except the numerical tables.
int plan_problem(const mcs_mesh* mesh, const mcs_options* opt, mcs_problem* pb) {
  const int d = mesh->dim;
  if (d != 2 && d != 3) {
    set_error("dim must be 2 or 3 (got %d)", d);
    return MCS_ERR_ARG;
  }
  const int k = opt->order;
  if (k < 2 || k > 5) {
    set_error("order k must be in 2..5 (got %d)", k);
    return k < 2 ? MCS_ERR_ARG : MCS_ERR_UNSUPPORTED;
  }
  if (mesh->n_vertices <= d || mesh->n_elements <= 0 || !mesh->vertices_host || !mesh->elements_host) {
    set_error("empty mesh");
    return MCS_ERR_ARG;
  }
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
  pb->sz = make_sizes(d, k);
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
    if (j - i == 1) {
      for (int c = 0; c < d; ++c) vbound[fl[i].v[c]] = 1;
    } else {
      int32_t g = (int32_t)free_fv.size();
      free_fv.push_back(fl[i].v);
      pb->h_facet_el.push_back(fl[i].e);
      pb->h_facet_el.push_back(fl[i + 1].e);
      pb->h_facet_slot.push_back(fl[i].slot);
      pb->h_facet_slot.push_back(fl[i + 1].slot);
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
    bool interior = true;
    for (int a = 0; a < d; ++a)
      if (c[a] == 0 || c[a] == pb->lattice[a] - 1) interior = false;
    if (interior != (vfree[v] >= 0)) {
      set_error("boundary of the mesh does not match the lattice boundary");
      return MCS_ERR_MESH;
    }
  }
  pb->mg.clear();
  {
    int n[3] = {pb->lattice[0] - 1, pb->lattice[1] - 1, d == 3 ? pb->lattice[2] - 1 : 0};
    while (true) {
      MGLevel L{};
      L.n[0] = n[0];
      L.n[1] = n[1];
      L.n[2] = n[2];
      L.nvert = (int64_t)(n[0] + 1) * (n[1] + 1) * (d == 3 ? n[2] + 1 : 1);
      L.nfree = (int64_t)(n[0] - 1) * (n[1] - 1) * (d == 3 ? n[2] - 1 : 1) * d;
      pb->mg.push_back(L);
      int nmin = std::min(n[0], n[1]);
      if (d == 3) nmin = std::min(nmin, n[2]);
      if (L.nfree <= pb->opt.coarse_max || nmin <= 2) break;
      for (int a = 0; a < d; ++a) n[a] = (int)coarse_count(n[a]) - 1;
    }
    const MGLevel& C = pb->mg.back();
    pb->nc = C.nfree;
    pb->h_cmap.clear();
    int N0 = C.n[0] + 1, N1 = C.n[1] + 1;
    for (int64_t v = 0; v < C.nvert; ++v) {
      int c[3] = {int(v % N0), int((v / N0) % N1), int(v / ((int64_t)N0 * N1))};
      bool interior = true;
      for (int a = 0; a < d; ++a)
        if (c[a] == 0 || c[a] == C.n[a]) interior = false;
      if (interior)
        for (int cc = 0; cc < d; ++cc) pb->h_cmap.push_back((int32_t)(v * d + cc));
    }
  }

  // ---- global layout
  pb->off_f = ne * s.nb;
  pb->off_p = pb->off_f + nff * s.nfb;
  pb->ndof = pb->off_p + ne * s.np;
  pb->np1 = nfv * d;
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
  L.add("colour_facets", I(nff));
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
  L.add("rD", Dd(r.D.size()));
  L.add("rBp", Dd(r.Bp.size()));
  L.add("rMp", Dd(r.Mp.size()));
  L.add("rMpinv", Dd(r.Mpinv.size()));
  L.add("rRf", Dd(r.Rf.size()));
  L.add("rcn", Dd(r.cn.size()));
  L.add("rct", Dd(r.ct.size()));
  L.add("rpconst", Dd(r.pconst.size()));
  L.add("rpmom", Dd(r.pmom.size()));
  L.add("rlatmap", I(r.latmap.size()));
  L.add("nu", Dd(ne));
  L.add("detJ", Dd(ne));
  L.add("Ad", Dd(ne * s.nd * s.nd));
  L.add("H", Dd(ne * s.nb * s.nd));
  L.add("Aoo", Dd(ne * s.nb * s.nb));
  L.add("Aooinv", Dd(ne * s.nb * s.nb));
  L.add("Ad32", Ff(ne * s.nd * s.nd));
  L.add("H32", Ff(ne * s.nb * s.nd));
  L.add("Aoo32", Ff(ne * s.nb * s.nb));
  L.add("Aooinv32", Ff(ne * s.nb * s.nb));
  L.add("Dinv", Dd(nff * s.nfb * s.nfb));
  L.add("EF", Dd(nff * s.nfb * d * d));
  L.add("Dinv32", Ff(nff * s.nfb * s.nfb));
  L.add("EF32", Ff(nff * s.nfb * d * d));
  L.add("W", Dd(ne * (d + 1) * d * s.nd));
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
  }
  L.add("Cinv", Dd(pb->nc * pb->nc));
  L.add("cmap", I(pb->nc));
  pb->n_slots = std::min<int64_t>(ne, 2048);
  pb->slot_doubles = (int64_t)s.nA * s.nsig + (int64_t)s.nlam * s.nsig * 2 + (int64_t)s.nA * s.nlam +
                     (int64_t)s.nA * s.nA + (int64_t)s.nlam * s.nlam + (int64_t)s.nb * s.nb * 2 + 64;
  L.add("cscratch", Dd(pb->n_slots * pb->slot_doubles));
  L.add("escr", Dd(ne * s.nd));
  L.add("escr2", Dd(ne * s.nd));
  L.add("fscr", Dd(nff * d * d));
  pb->nred = 4096;
  L.add("red", Dd(pb->nred));
  L.add("scal", Dd(256));
  pb->nvec64 = 24;
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
