// C ABI of the MCS solver: plan / bind / condense / load / apply /
// precond_apply / solve.  Host orchestration of the kernels:
//   K-hat^{-1} (eq. mhatinvfactor) with two A-hat_ext^{-1} applications
//   (Sec. 6.1), A-hat^d_m^{-1} (Corollary aux_pc_mult: forward coloured block
//   Gauss-Seidel sweeps, coarse correction E^d C^{-1} E^d^T, backward sweeps),
//   C = one V(1,1) cycle on the P1 lattice hierarchy, and preconditioned MINRES
//   (Paige-Saunders) on K (eq. femSPmat), optionally in FP32 inside FP64
//   iterative refinement.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "ctx.h"

namespace mcs {
int plan_problem(const mcs_mesh* mesh, const mcs_options* opt, mcs_problem* pb);
int layout_workspace(mcs_problem* pb);
int64_t offset_of(const mcs_problem* pb, const char* name);
const char* last_error();
}  // namespace mcs

using namespace mcs;

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) {                                                               \
      set_error("HIP error '%s' at %s:%d", hipGetErrorString(e_), __FILE__, __LINE__);   \
      return MCS_ERR_HIP;                                                                 \
    }                                                                                     \
  } while (0)

// Reduction scratch of mcs_solve_rhs_noalloc: the dot products' partial sums
// (at most 1024), their scalar slot and the pressure mean.  Each device holds
// its own copy until the process ends; host code uses only the device address
// that hipGetSymbolAddress returns for it (noalloc_scratch_ptr).
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = 4096;   // 32 KiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static double* noalloc_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

namespace {

// Looks up the device address of `scratch` on the current device, once per
// device (called by mcs_bind with the problem's device current).
int noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
    set_error("device %d outside the no-alloc scratch table", device);
    return MCS_ERR_ARG;
  }
  if (noalloc_scratch_ptr[device]) return MCS_OK;
  void* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  noalloc_scratch_ptr[device] = static_cast<double*>(ptr);
  return MCS_OK;
}

// Smoother launch-shape tuner: times every candidate shape on the largest
// colour (scratch vectors, one warm-up and three timed launches) and keeps the
// fastest for work precision R.
template <typename R>
int tune_smoother_precision(mcs_problem* pb, int slot) {
  Ctx<R> c(pb);
  int best_col = -1;
  int64_t nbest = 0;
  for (int col = 0; col < pb->ncol; ++col) {
    const int64_t n = pb->colour_off[col + 1] - pb->colour_off[col];
    if (n > nbest) {
      nbest = n;
      best_col = col;
    }
  }
  if (best_col < 0) return MCS_OK;
  hipStream_t st = c.st;
  R* x = c.v(PT);
  R* sv = c.v(PS);
  R* y = c.escr;
  launch_fill<R>(st, c.n, R(0), x);
  launch_fill<R>(st, c.n, R(0), sv);
  launch_fill<R>(st, pb->ne * pb->sz.nd, R(0), y);
  const int T1 = smooth_team_threads(pb->sz.nd);
  std::vector<std::pair<int, int64_t>> cand;
  for (int fpw : {1, 2}) {
    if (fpw == 2 && 2 * T1 > 512) continue;
    for (int64_t cap : {int64_t(0), int64_t(2048), int64_t(4096), int64_t(8192)}) cand.push_back({fpw, cap});
  }
  struct Events {  // released on every return path
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      ApiLock lock(device_api_mutex());
      for (auto x : e)
        if (x) hipEventDestroy(x);
    }
  } ev;
  {
    ApiLock lock(device_api_mutex());
    HIPCHK(hipEventCreate(&ev.e[0]));
    HIPCHK(hipEventCreate(&ev.e[1]));
  }
  hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
  const int32_t c0 = pb->colour_off[best_col], c1 = pb->colour_off[best_col + 1];
  double best = 1e300;
  for (auto& cf : cand) {
    launch_smooth_phase<R>(st, c.P, c.O, c0, c1, x, sv, y, cf.first, cf.second);
    HIPCHK(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) launch_smooth_phase<R>(st, c.P, c.O, c0, c1, x, sv, y, cf.first, cf.second);
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    const double us = ms * 1e3 / 3.0;
    if (us < best) {
      best = us;
      pb->tune_fpw[slot] = cf.first;
      pb->tune_cap[slot] = cf.second;
      pb->tune_us[slot] = us;
    }
  }
  return MCS_OK;
}

// Operator apply tuner: times K x (the apply of the iteration) with the
// numbers of A^d rows per thread (4 only in FP32; plain storage only: the
// split FP64 storage takes one row per thread) whose H products use the lane
// width of the default choice, so that every candidate gives bitwise the same
// results, and keeps the fastest.
template <typename R>
int tune_apply_precision(mcs_problem* pb, int slot) {
  const int nd = pb->sz.nd;
  const int cp0 = (sizeof(R) == 4 && nd % 4 == 0) ? 4 : nd % 2 == 0 ? 2 : 1;   // the default
  std::vector<int> cand;
  for (int cp : {1, 2, 4})
    if (cp <= cp0 && nd % cp == 0 && apply_h_lanes(nd, cp) == apply_h_lanes(nd, cp0) &&
        apply_col_split(nd, cp) == apply_col_split(nd, cp0))
      cand.push_back(cp);
  if (cand.empty()) return MCS_OK;   // (a single choice is still timed, for the record)
  if (pb->sz.nb == 0 && pb->sz.np == 1) return MCS_OK;   // k = 1: one wave per element, no rows to choose
  if (sizeof(R) == 8 && pb->lean) return MCS_OK;         // split storage: one row per thread
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      ApiLock lock(device_api_mutex());
      for (auto x : e)
        if (x) hipEventDestroy(x);
    }
  } ev;
  {
    ApiLock lock(device_api_mutex());
    HIPCHK(hipEventCreate(&ev.e[0]));
    HIPCHK(hipEventCreate(&ev.e[1]));
  }
  double best = 1e300;
  int best_rpt = 0;
  for (int rpt : cand) {
    pb->tune_rpt[slot] = rpt;
    Ctx<R> c(pb);
    R* x = c.v(PT);
    R* y = c.v(PS);
    launch_fill<R>(c.st, c.n, R(1), x);
    c.apply(x, y, 1 | 2 | 4);
    HIPCHK(hipEventRecord(ev.e[0], c.st));
    for (int r = 0; r < 3; ++r) c.apply(x, y, 1 | 2 | 4);
    HIPCHK(hipEventRecord(ev.e[1], c.st));
    HIPCHK(hipEventSynchronize(ev.e[1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    const double us = ms * 1e3 / 3.0;
    if (us < best) {
      best = us;
      best_rpt = rpt;
    }
  }
  pb->tune_rpt[slot] = best_rpt;
  pb->tune_rpt_us[slot] = best;
  return MCS_OK;
}

// Tunes each precision slot once per plan, except the slots whose shape the
// caller fixed with mcs_set_launch_config / mcs_set_apply_config.
int tune_smoother(mcs_problem* pb) {
  int rc = MCS_OK;
  if (!pb->lean && !pb->tune_fixed[0] && pb->tune_us[0] == 0.0) rc = tune_smoother_precision<double>(pb, 0);
  if (rc) return rc;
  if (!pb->tune_fixed[1] && pb->tune_us[1] == 0.0) rc = tune_smoother_precision<float>(pb, 1);
  if (rc) return rc;
  if (!pb->tune_rpt_fixed[0] && pb->tune_rpt_us[0] == 0.0) rc = tune_apply_precision<double>(pb, 0);
  if (rc) return rc;
  if (pb->opt.precision == 1 && !pb->tune_rpt_fixed[1] && pb->tune_rpt_us[1] == 0.0)
    rc = tune_apply_precision<float>(pb, 1);
  return rc;
}

int check_bound(mcs_problem* pb) {
  if (!pb) {
    set_error("null problem");
    return MCS_ERR_ARG;
  }
  if (!pb->ws) {
    set_error("problem is not bound to a workspace");
    return MCS_ERR_STATE;
  }
  return MCS_OK;
}

int sync_status(mcs_problem* pb, const char* what) {
  HIPCHK(hipStreamSynchronize(pb->stream));
  HIPCHK(hipGetLastError());
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, pb->p.scal + 200, sizeof(int), hipMemcpyDeviceToHost, pb->stream));
  HIPCHK(hipStreamSynchronize(pb->stream));
  if (st & 8) {
    set_error("%s: viscosity must be positive and finite", what);
    return MCS_ERR_ARG;
  }
  if (st & 7) {
    set_error("%s: Cholesky breakdown (code %d: 1 element, 2 facet block, 4 coarse grid)", what, st);
    return MCS_ERR_NOT_SPD;
  }
  return MCS_OK;
}

}  // namespace

extern "C" {

const char* mcs_status_string(int status) {
  switch (status) {
    case MCS_OK: return "ok";
    case MCS_ERR_ARG: return "invalid argument";
    case MCS_ERR_MESH: return "invalid mesh";
    case MCS_ERR_WORKSPACE: return "workspace missing or too small";
    case MCS_ERR_NOT_SPD: return "Cholesky breakdown (matrix not SPD)";
    case MCS_ERR_NOT_CONVERGED: return "not converged";
    case MCS_ERR_BREAKDOWN: return "MINRES breakdown";
    case MCS_ERR_NONFINITE: return "non-finite value";
    case MCS_ERR_STATE: return "call out of order";
    case MCS_ERR_HIP: return "HIP runtime error";
    case MCS_ERR_UNSUPPORTED: return "unsupported order or dimension";
    default: return "unknown status";
  }
}

const char* mcs_last_error(void) { return last_error(); }

int mcs_plan(const mcs_mesh* mesh, const mcs_options* options, mcs_problem** out, mcs_info* info) {
  if (!mesh || !options || !out) {
    set_error("null argument");
    return MCS_ERR_ARG;
  }
  *out = nullptr;
  mcs_problem* pb = new (std::nothrow) mcs_problem();
  if (!pb) {
    set_error("out of host memory");
    return MCS_ERR_ARG;
  }
  int rc;
  try {
    rc = plan_problem(mesh, options, pb);
    if (rc == MCS_OK) {
      pb->ref = build_ref_tables(pb->d, pb->sz.k);
      rc = layout_workspace(pb);
    }
  } catch (const std::exception& ex) {
    set_error("plan failed: %s", ex.what());
    rc = MCS_ERR_ARG;
  }
  if (rc != MCS_OK) {
    delete pb;
    return rc;
  }
  if (info) {
    const Sizes& s = pb->sz;
    info->n_dof = pb->ndof;
    info->n_bubble_dofs = pb->off_f;
    info->n_facet_dofs = pb->off_p - pb->off_f;
    info->n_pressure_dofs = pb->ndof - pb->off_p;
    info->n_p1_dofs = pb->np1;
    info->off_facet = pb->off_f;
    info->off_pressure = pb->off_p;
    info->n_bub = s.nb;
    info->n_F = s.nF;
    info->n_hat = s.nh;
    info->n_fb = s.nfb;
    info->n_p = s.np;
    info->n_lat = s.nlat;
    info->n_free_facets = (int32_t)pb->nff;
    info->n_colours = pb->ncol;
    info->n_mg_levels = (int32_t)pb->mg.size();
    info->workspace_bytes = pb->ws_bytes;
  }
  *out = pb;
  return MCS_OK;
}

int mcs_bind(mcs_problem* pb, void* workspace, size_t bytes, void* stream) {
  ApiLock lock(device_api_mutex());
  if (!pb) {
    set_error("null problem");
    return MCS_ERR_ARG;
  }
  if (!workspace || bytes < pb->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
    set_error("workspace must be >= %zu bytes and 256-byte aligned", pb->ws_bytes);
    return MCS_ERR_WORKSPACE;
  }
  HIPCHK(hipGetDevice(&pb->device));
  {
    int rc = noalloc_scratch_init(pb->device);
    if (rc) return rc;
  }
  pb->ws = workspace;
  pb->stream = static_cast<hipStream_t>(stream);
  pb->condensed = false;
  DevPtrs& p = pb->p;
  p.elem_ff = ws_ptr<int32_t>(pb, "elem_ff");
  p.elem_verts = ws_ptr<int32_t>(pb, "elem_verts");
  p.elem_perm = ws_ptr<int32_t>(pb, "elem_perm");
  p.facet_el = ws_ptr<int32_t>(pb, "facet_el");
  p.facet_slot = ws_ptr<int32_t>(pb, "facet_slot");
  p.facet_out = ws_ptr<int32_t>(pb, "facet_out");
  p.xD = ws_ptr<double>(pb, "xD");
  p.colour_desc = ws_ptr<int32_t>(pb, "colour_desc");
  p.facet_vfree = ws_ptr<int32_t>(pb, "facet_vfree");
  p.vinc_off = ws_ptr<int32_t>(pb, "vinc_off");
  p.vinc = ws_ptr<int32_t>(pb, "vinc");
  p.vert_elem_off = ws_ptr<int32_t>(pb, "vert_elem_off");
  p.vert_elem = ws_ptr<int32_t>(pb, "vert_elem");
  p.coords = ws_ptr<double>(pb, "coords");
  p.vfree_of_lat = ws_ptr<int32_t>(pb, "vfree_of_lat");
  p.free_to_lat = ws_ptr<int32_t>(pb, "free_to_lat");
  p.rV = ws_ptr<double>(pb, "rV");
  p.rBf = ws_ptr<double>(pb, "rBf");
  p.rU = ws_ptr<double>(pb, "rU");
  p.rL = ws_ptr<double>(pb, "rL");
  p.rLam = ws_ptr<double>(pb, "rLam");
  p.rD = ws_ptr<double>(pb, "rD");
  p.rBp = ws_ptr<double>(pb, "rBp");
  p.rMp = ws_ptr<double>(pb, "rMp");
  p.rMpinv = ws_ptr<double>(pb, "rMpinv");
  p.rRf = ws_ptr<double>(pb, "rRf");
  p.rcn = ws_ptr<double>(pb, "rcn");
  p.rct = ws_ptr<double>(pb, "rct");
  p.rpconst = ws_ptr<double>(pb, "rpconst");
  p.rpmom = ws_ptr<double>(pb, "rpmom");
  p.rphi = ws_ptr<double>(pb, "rphi");
  p.rpidx = ws_ptr<double>(pb, "rpidx");
  p.rpsi = ws_ptr<double>(pb, "rpsi");
  p.rpsib = ws_ptr<double>(pb, "rpsib");
  p.rlatmap = ws_ptr<int32_t>(pb, "rlatmap");
  p.nu = ws_ptr<double>(pb, "nu");
  p.detJ = ws_ptr<double>(pb, "detJ");
  p.Ad = ws_ptr<double>(pb, "Ad");
  p.H = ws_ptr<double>(pb, "H");
  p.Aoo = ws_ptr<double>(pb, "Aoo");
  p.Aooinv = ws_ptr<double>(pb, "Aooinv");
  p.Ad32 = ws_ptr<float>(pb, "Ad32");
  p.H32 = ws_ptr<float>(pb, "H32");
  p.Aoo32 = ws_ptr<float>(pb, "Aoo32");
  p.Aooinv32 = ws_ptr<float>(pb, "Aooinv32");
  p.Dinv = ws_ptr<double>(pb, "Dinv");
  p.EF = ws_ptr<double>(pb, "EF");
  p.Dinv32 = ws_ptr<float>(pb, "Dinv32");
  p.DinvP = ws_ptr<double>(pb, "DinvP");
  p.DinvP32 = ws_ptr<float>(pb, "DinvP32");
  p.EF32 = ws_ptr<float>(pb, "EF32");
  p.W = ws_ptr<double>(pb, "W");
  p.W32 = ws_ptr<float>(pb, "W32");
  p.Adl = ws_ptr<float>(pb, "Adl");
  p.Hl = ws_ptr<float>(pb, "Hl");
  p.Aool = ws_ptr<float>(pb, "Aool");
  p.adtmp = ws_ptr<double>(pb, "adtmp");
  p.Cinv = ws_ptr<double>(pb, "Cinv");
  p.cmap = ws_ptr<int32_t>(pb, "cmap");
  p.cscratch = ws_ptr<double>(pb, "cscratch");
  p.escr = ws_ptr<double>(pb, "escr");
  p.escr2 = ws_ptr<double>(pb, "escr2");
  p.fscr = ws_ptr<double>(pb, "fscr");
  p.red = ws_ptr<double>(pb, "red");
  p.scal = ws_ptr<double>(pb, "scal");
  p.wcount = ws_ptr<unsigned long long>(pb, "wcount");
  p.blk_el = ws_ptr<int32_t>(pb, "blk_el");
  p.blk_slot = ws_ptr<int32_t>(pb, "blk_slot");
  p.blk_g = ws_ptr<int32_t>(pb, "blk_g");
  p.colour_blocks = ws_ptr<int32_t>(pb, "colour_blocks");
  p.Afull = ws_ptr<double>(pb, "Afull");
  p.Binv = ws_ptr<double>(pb, "Binv");
  p.Wfull = ws_ptr<double>(pb, "Wfull");
  p.Eo = ws_ptr<double>(pb, "Eo");
  p.Eoref = ws_ptr<double>(pb, "Eoref");
  p.yfull = ws_ptr<double>(pb, "yfull");
  p.eto = ws_ptr<double>(pb, "eto");
  p.vec = ws_ptr<double>(pb, "vec");
  p.vec32 = ws_ptr<float>(pb, "vec32");
  p.p1 = ws_ptr<double>(pb, "p1");
  p.p132 = ws_ptr<float>(pb, "p132");

  hipStream_t st = pb->stream;
  auto up = [&](void* dst, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st);
  };
  const RefTables& r = pb->ref;
  HIPCHK(up(p.elem_ff, pb->h_elem_ff.data(), pb->h_elem_ff.size() * 4));
  HIPCHK(up(p.elem_verts, pb->h_elem_verts.data(), pb->h_elem_verts.size() * 4));
  HIPCHK(up(p.elem_perm, pb->h_elem_perm.data(), pb->h_elem_perm.size() * 4));
  HIPCHK(up(p.facet_el, pb->h_facet_el.data(), pb->h_facet_el.size() * 4));
  HIPCHK(up(p.facet_slot, pb->h_facet_slot.data(), pb->h_facet_slot.size() * 4));
  HIPCHK(up(p.facet_out, pb->h_facet_out.data(), pb->h_facet_out.size() * 4));
  {
    // colour-ordered facet records, so that a smoother team finds both
    // neighbours of its facet with one load
    std::vector<int32_t> desc(pb->h_colour_facets.size() * 4);
    for (size_t i = 0; i < pb->h_colour_facets.size(); ++i) {
      const int32_t g = pb->h_colour_facets[i];
      desc[4 * i] = g;
      desc[4 * i + 1] = pb->h_facet_el[2 * g];
      desc[4 * i + 2] = pb->h_facet_el[2 * g + 1];
      desc[4 * i + 3] = (pb->h_facet_slot[2 * g] & 0xFF) | ((pb->h_facet_slot[2 * g + 1] & 0xFF) << 8);
    }
    HIPCHK(up(p.colour_desc, desc.data(), desc.size() * 4));
    HIPCHK(hipStreamSynchronize(st));
  }
  HIPCHK(up(p.facet_vfree, pb->h_facet_vfree.data(), pb->h_facet_vfree.size() * 4));
  HIPCHK(up(p.vinc_off, pb->h_vinc_off.data(), pb->h_vinc_off.size() * 4));
  HIPCHK(up(p.vinc, pb->h_vinc.data(), pb->h_vinc.size() * 4));
  HIPCHK(up(p.vert_elem_off, pb->h_vert_elem_off.data(), pb->h_vert_elem_off.size() * 4));
  HIPCHK(up(p.vert_elem, pb->h_vert_elem.data(), pb->h_vert_elem.size() * 4));
  HIPCHK(up(p.coords, pb->h_coords.data(), pb->h_coords.size() * 8));
  HIPCHK(up(p.vfree_of_lat, pb->h_vfree_of_lat.data(), pb->h_vfree_of_lat.size() * 4));
  HIPCHK(up(p.free_to_lat, pb->h_free_to_lat.data(), pb->h_free_to_lat.size() * 4));
  HIPCHK(up(p.rV, r.V.data(), r.V.size() * 8));
  HIPCHK(up(p.rBf, r.Bf.data(), r.Bf.size() * 8));
  HIPCHK(up(p.rU, r.U.data(), r.U.size() * 8));
  HIPCHK(up(p.rL, r.L.data(), r.L.size() * 8));
  HIPCHK(up(p.rLam, r.Lam.data(), r.Lam.size() * 8));
  HIPCHK(up(p.rD, r.D.data(), r.D.size() * 8));
  HIPCHK(up(p.rBp, r.Bp.data(), r.Bp.size() * 8));
  HIPCHK(up(p.rMp, r.Mp.data(), r.Mp.size() * 8));
  HIPCHK(up(p.rMpinv, r.Mpinv.data(), r.Mpinv.size() * 8));
  HIPCHK(up(p.rRf, r.Rf.data(), r.Rf.size() * 8));
  HIPCHK(up(p.rcn, r.cn.data(), r.cn.size() * 8));
  HIPCHK(up(p.rct, r.ct.data(), r.ct.size() * 8));
  HIPCHK(up(p.rpconst, r.pconst.data(), r.pconst.size() * 8));
  HIPCHK(up(p.rpmom, r.pmom.data(), r.pmom.size() * 8));
  HIPCHK(up(p.rphi, r.phi.data(), r.phi.size() * 8));
  HIPCHK(up(p.rpidx, r.pidx.data(), r.pidx.size() * 8));
  HIPCHK(up(p.rpsi, r.psi.data(), r.psi.size() * 8));
  HIPCHK(up(p.rpsib, r.psib.data(), r.psib.size() * 8));
  HIPCHK(up(p.rlatmap, r.latmap.data(), r.latmap.size() * 4));
  HIPCHK(up(p.cmap, pb->h_cmap.data(), pb->h_cmap.size() * 4));
  if (p.blk_el) {
    HIPCHK(up(p.blk_el, pb->h_blk_el.data(), pb->h_blk_el.size() * 4));
    HIPCHK(up(p.blk_slot, pb->h_blk_slot.data(), pb->h_blk_slot.size() * 4));
    HIPCHK(up(p.blk_g, pb->h_blk_g.data(), pb->h_blk_g.size() * 4));
    HIPCHK(up(p.colour_blocks, pb->h_colour_blocks.data(), pb->h_colour_blocks.size() * 4));
    HIPCHK(up(p.Eoref, r.Eo.data(), r.Eo.size() * 8));
  }
  // multigrid lattice vectors start (and stay) zero on the boundary; block tables
  const int d = pb->d;
  for (auto& M : pb->mg) {
    char* base = static_cast<char*>(pb->ws);
    std::vector<MGBlockDev> tab(M.blocks.size());
    for (size_t j = 0; j < M.blocks.size(); ++j) {
      const MGBlock& B = M.blocks[j];
      MGBlockDev& T = tab[j];
      for (int a = 0; a < 3; ++a) {
        T.n[a] = B.n[a];
        T.nc3[a] = B.nc3[a];
      }
      T.prob = B.prob;
      T.ffm = B.ffm;
      T.voff = B.voff;
      T.nvert = B.nvert;
      T.cvoff = B.cvoff;
      T.nvert_c = B.nvert_c;
      T.nc = B.nc;
      T.cmap_off = B.cmap_off;
      T.cinv_off = B.cinv_off;
    }
    HIPCHK(up(base + M.off_blk, tab.data(), tab.size() * sizeof(MGBlockDev)));
    HIPCHK(hipStreamSynchronize(st));   // tab is a local host buffer
    HIPCHK(hipMemsetAsync(base + M.off_x, 0, (size_t)M.nvert * d * 8, st));
    HIPCHK(hipMemsetAsync(base + M.off_b, 0, (size_t)M.nvert * d * 8, st));
    HIPCHK(hipMemsetAsync(base + M.off_r, 0, (size_t)M.nvert * d * 8, st));
  }
  HIPCHK(hipMemsetAsync(p.scal, 0, 256 * 8, st));
  HIPCHK(hipStreamSynchronize(st));
  return MCS_OK;
}

// Geometry, reference tables, viscosity and slot scratch of the element kernels.
static CondParams cond_params(mcs_problem* pb, int* status) {
  DevPtrs& p = pb->p;
  CondParams C{};
  C.s = pb->sz;
  C.ne = pb->ne;
  C.slot_doubles = pb->slot_doubles;
  C.elem_verts = p.elem_verts;
  C.coords = p.coords;
  C.nu = p.nu;
  C.rV = p.rV;
  C.rBf = p.rBf;
  C.rU = p.rU;
  C.rL = p.rL;
  C.rLam = p.rLam;
  C.rD = p.rD;
  for (int f = 0; f < 4; ++f) C.facet_measure[f] = pb->ref.facet_measure[f];
  C.scratch = p.cscratch;
  C.detJ = p.detJ;
  C.status = status;
  C.elem_ff = p.elem_ff;
  C.facet_out = pb->has_outlet ? p.facet_out : nullptr;
  return C;
}

int mcs_condense(mcs_problem* pb, const double* nu) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!nu) {
    set_error("null viscosity");
    return MCS_ERR_ARG;
  }
  hipStream_t st = pb->stream;
  DevPtrs& p = pb->p;
  int* status = reinterpret_cast<int*>(p.scal + 200);
  HIPCHK(hipMemsetAsync(status, 0, sizeof(int), st));
  HIPCHK(hipMemcpyAsync(p.nu, nu, pb->ne * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_check_nu(st, p.nu, pb->ne, status);
  rc = sync_status(pb, "condense");
  if (rc) return rc;

  CondParams C = cond_params(pb, status);
  C.Ad = p.Ad;
  C.H = p.H;
  C.Aoo = p.Aoo;
  C.Aooinv = p.Aooinv;
  C.Ad32 = p.Ad32;
  C.H32 = p.H32;
  C.Aoo32 = p.Aoo32;
  C.Aooinv32 = p.Aooinv32;
  C.Adl = p.Adl;
  C.Hl = p.Hl;
  C.Aool = p.Aool;
  C.adtmp = p.adtmp;
  C.adtmp_stride = (int64_t)pb->sz.nd * pb->sz.nd;
  C.Afull = p.Afull;
  launch_condense(st, C, (int)pb->n_slots);

  FacetSetupParams F{};
  F.s = pb->sz;
  F.nff = pb->nff;
  F.facet_el = p.facet_el;
  F.facet_slot = p.facet_slot;
  F.elem_verts = p.elem_verts;
  F.coords = p.coords;
  F.Ad = p.Ad;
  F.Adh = p.Ad32;
  F.Adl = p.Adl;
  F.facet_out = pb->has_outlet ? p.facet_out : nullptr;
  F.rcn = p.rcn;
  F.rct = p.rct;
  F.Dinv = p.Dinv;
  F.Dinv32 = p.Dinv32;
  F.DinvP = p.DinvP;
  F.DinvP32 = p.DinvP32;
  F.EF = p.EF;
  F.EF32 = p.EF32;
  F.status = status;
  F.elem_ff = p.elem_ff;
  if (pb->opt.smoother == 3 && pb->nff > 0) {
    // the facet blocks become M_F = D_F + diag(l_F) (l1-Jacobi); the FP64
    // refinement slots are free during the condensation
    Ctx<double> c(pb);
    double* diag = c.v(VR64) + pb->off_f;
    double* l1 = c.v(VT64) + pb->off_f;
    launch_l1_terms(st, F, diag, l1);
    F.l1diag = l1;
  }
  if (pb->nff > 0) launch_facet_setup(st, F);
  launch_wsetup(st, F, p.elem_ff, pb->ne, p.W, p.W32);
  if (pb->opt.smoother == 2) {
    Ctx<double> c(pb);
    launch_full_setup(st, pb->sz, pb->ne, c.full_dev(), p.elem_verts, p.coords, p.elem_ff, p.EF, status);
  }

  // P1 multigrid hierarchy
  const int d = pb->d, stn = d == 3 ? 27 : 9;
  char* base = static_cast<char*>(pb->ws);
  P1Params A{};
  A.d = d;
  A.nblk = (int)pb->mg[0].blocks.size();
  A.blk = reinterpret_cast<const MGBlockDev*>(base + pb->mg[0].off_blk);
  A.maxv = 0;
  for (auto& B : pb->mg[0].blocks) A.maxv = std::max(A.maxv, B.nvert);
  A.vert_elem_off = p.vert_elem_off;
  A.vert_elem = p.vert_elem;
  A.elem_verts = p.elem_verts;
  A.coords = p.coords;
  A.nu = p.nu;
  A.A = reinterpret_cast<double*>(base + pb->mg[0].off_A);
  A.k = pb->sz.k;
  A.penalty = OUTLET_PENALTY;
  launch_p1_assemble(st, A);
  const int64_t scratch_doubles = pb->n_slots * pb->slot_doubles;
  for (size_t l = 0; l < pb->mg.size(); ++l) {
    MGLevel& M = pb->mg[l];
    MGSetupParams S{};
    S.d = d;
    S.nblk = (int)M.blocks.size();
    S.ncont = M.ncont;
    S.blk = reinterpret_cast<const MGBlockDev*>(base + M.off_blk);
    S.maxv = M.maxv;
    S.maxvc = M.maxvc;
    S.maxnc = M.maxnc;
    S.A = reinterpret_cast<double*>(base + M.off_A);
    S.Dinv = reinterpret_cast<double*>(base + M.off_Dinv);
    S.Dinv32 = reinterpret_cast<float*>(base + M.off_Dinv + (size_t)M.nvert * d * d * 8);
    S.cmap = p.cmap;
    size_t nA = (size_t)M.nvert * stn * d * d;
    if (M.ncont > 0) {
      S.Ac = reinterpret_cast<double*>(base + pb->mg[l + 1].off_A);
      launch_mg_l1(st, S);
      launch_mg_rap(st, S);
    }
    // dense coarsest solves, in chunks whose matrices and Cholesky workspaces
    // fit the condensation scratch
    for (int j0 = M.ncont; j0 < S.nblk;) {
      const int64_t base_off = M.blocks[j0].cinv_off;
      int j1 = j0;
      while (j1 < S.nblk && 2 * (M.blocks[j1].cinv_off + M.blocks[j1].nc * M.blocks[j1].nc - base_off) <= scratch_doubles)
        ++j1;
      if (j1 == j0) {
        set_error("coarsest level too large for the scratch area");
        return MCS_ERR_WORKSPACE;
      }
      launch_coarse(st, S, j0 - M.ncont, j1 - j0, base_off, p.cscratch, p.Cinv, status);
      j0 = j1;
    }
    launch_to_f32(st, reinterpret_cast<double*>(base + M.off_A),
                  reinterpret_cast<float*>(base + M.off_A + nA * 8), (int64_t)nA);
  }
  rc = sync_status(pb, "condense");
  if (rc) return rc;
  if (pb->opt.autotune) {   // once per plan and slot; later condensations reuse the shapes
    rc = tune_smoother(pb);
    if (rc) return rc;
  }
  pb->condensed = true;
  return MCS_OK;
}

int mcs_load(mcs_problem* pb, const double* f_lattice, double* b) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_load needs mcs_condense first");
    return MCS_ERR_STATE;
  }
  if (!f_lattice || !b) {
    set_error("null argument");
    return MCS_ERR_ARG;
  }
  hipStream_t st = pb->stream;
  DevPtrs& p = pb->p;
  CondParams C{};
  C.s = pb->sz;
  C.ne = pb->ne;
  C.elem_verts = p.elem_verts;
  C.coords = p.coords;
  SolveParams P = solve_params(pb);
  launch_fill<double>(st, pb->ndof, 0.0, b);
  launch_load(st, C, P, p.elem_perm, p.rlatmap, p.rRf, f_lattice, b, p.escr);
  launch_facet_sum<double>(st, P, p.escr, nullptr, 1.0, b);
  if (pb->has_dirichlet) {
    // lifted Dirichlet data: b -= K (0 + x_D)
    Ctx<double> c(pb);
    c.P.xD = p.xD;
    double *z = c.v(VT64), *kz = c.v(VR64);
    launch_fill<double>(st, pb->ndof, 0.0, z);
    c.apply(z, kz, 1 | 2 | 4);
    launch_axpby<double>(st, pb->ndof, -1.0, kz, 1.0, b);
  }
  HIPCHK(hipGetLastError());
  return MCS_OK;
}

int mcs_set_dirichlet(mcs_problem* pb, const double* g_lattice_host) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!g_lattice_host) {
    pb->has_dirichlet = false;
    return MCS_OK;
  }
  std::vector<double> xd;
  try {
    dirichlet_lift(pb, g_lattice_host, xd);
  } catch (const std::exception& ex) {
    set_error("mcs_set_dirichlet: %s", ex.what());
    return MCS_ERR_ARG;
  }
  for (double v : xd)
    if (!std::isfinite(v)) {
      set_error("mcs_set_dirichlet: non-finite boundary data");
      return MCS_ERR_ARG;
    }
  HIPCHK(hipMemcpyAsync(pb->p.xD, xd.data(), xd.size() * 8, hipMemcpyHostToDevice, pb->stream));
  HIPCHK(hipStreamSynchronize(pb->stream));
  pb->has_dirichlet = true;
  return MCS_OK;
}

}  // extern "C"

namespace {

template <typename R>
int apply_op(mcs_problem* pb, int op, const void* xv, void* yv) {
  Ctx<R> c(pb);
  const R* x = static_cast<const R*>(xv);
  R* y = static_cast<R*>(yv);
  switch (op) {
    case MCS_OP_K: c.apply(x, y, 1 | 2 | 4); break;
    case MCS_OP_A: c.apply(x, y, 1 | 16); break;
    case MCS_OP_ADELTA: c.apply(x, y, 1 | 8); break;
    case MCS_OP_B: c.apply(x, y, 4 | 16); break;
    case MCS_OP_BT: c.apply(x, y, 2 | 16); break;
    default:
      set_error("unknown operator %d", op);
      return MCS_ERR_ARG;
  }
  HIPCHK(hipGetLastError());
  return MCS_OK;
}

template <typename R>
int precond_op(mcs_problem* pb, int op, const void* rv, void* zv) {
  Ctx<R> c(pb);
  const R* r = static_cast<const R*>(rv);
  R* z = static_cast<R*>(zv);
  const int d = pb->d;
  switch (op) {
    case MCS_PC_KHAT: c.khat(r, z); break;
    case MCS_PC_AEXT: c.ext_inv(r, z); break;
    case MCS_PC_ADELTA_MULT: c.ad_inv(r, z); break;
    case MCS_PC_SMOOTH_FWD:
    case MCS_PC_SMOOTH_BWD:
      launch_fill<R>(c.st, c.n, R(0), z);
      launch_fill<R>(c.st, pb->ne * pb->sz.nd, R(0), c.escr);
      c.sweeps(z, r, c.escr, op == MCS_PC_SMOOTH_FWD);
      break;
    case MCS_PC_AUX:
      launch_fill<R>(c.st, c.n, R(0), z);
      c.aux(r, z, 1);
      break;
    case MCS_PC_EDELTA:
      launch_fill<R>(c.st, c.n, R(0), z);
      launch_ed<R>(c.st, c.P, c.O, pb->p.facet_vfree, pb->p.free_to_lat, r, z, 0, 1);
      break;
    case MCS_PC_EDELTA_T:
      launch_edt<R>(c.st, c.P, c.O, r, c.fscr, pb->nfv, pb->p.vinc_off, pb->p.vinc, pb->p.free_to_lat, z, 1);
      break;
    case MCS_PC_MG: {
      R* b0 = (R*)c.L[0].b;
      R* x0 = (R*)c.L[0].x;
      launch_scatter_compact<R>(c.st, pb->nfv, d, pb->p.free_to_lat, r, b0);
      c.vcycle(0);
      launch_gather_compact<R>(c.st, pb->nfv, d, pb->p.free_to_lat, x0, z);
      break;
    }
    case MCS_PC_MP_INV:
      launch_fill<R>(c.st, c.n, R(0), z);
      c.elem_press(r, r, z, 0);
      break;
    default:
      set_error("unknown preconditioner operator %d", op);
      return MCS_ERR_ARG;
  }
  HIPCHK(hipGetLastError());
  return MCS_OK;
}
}  // namespace

extern "C" {

int mcs_apply(mcs_problem* pb, int op, int dt, const void* x, void* y) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_apply needs mcs_condense first");
    return MCS_ERR_STATE;
  }
  if (!x || !y) {
    set_error("null vector");
    return MCS_ERR_ARG;
  }
  if (dt == MCS_F64) return apply_op<double>(pb, op, x, y);
  if (dt == MCS_F32) return apply_op<float>(pb, op, x, y);
  set_error("unknown dtype %d", dt);
  return MCS_ERR_ARG;
}

int mcs_precond_apply(mcs_problem* pb, int op, int dt, const void* r, void* z) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_precond_apply needs mcs_condense first");
    return MCS_ERR_STATE;
  }
  if (!r || !z) {
    set_error("null vector");
    return MCS_ERR_ARG;
  }
  if (dt == MCS_F64) {
    if (pb->lean) {
      set_error("precision 1 keeps the preconditioner in FP32 only");
      return MCS_ERR_STATE;
    }
    return precond_op<double>(pb, op, r, z);
  }
  if (dt == MCS_F32) return precond_op<float>(pb, op, r, z);
  set_error("unknown dtype %d", dt);
  return MCS_ERR_ARG;
}

int mcs_normalize_pressure(mcs_problem* pb, double* x) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_normalize_pressure needs mcs_condense first");
    return MCS_ERR_STATE;
  }
  if (pb->has_outlet) return MCS_OK;   // p is unique with an outlet
  SolveParams P = solve_params(pb);
  launch_pressure_mean(pb->stream, P, pb->p.rpmom, pb->p.rpconst, x, pb->p.red);
  HIPCHK(hipGetLastError());
  return MCS_OK;
}

// The iteration of mcs_solve_rhs.  Dot products reduce into `red` (>= 1024
// partial sums) and leave their scalar in host memory: written directly
// through host_dev (device alias of pinned memory) when it is given, else in
// `scal` and copied into *host.  The pressure mean reduces into `red` too.
static int solve_rhs_run(mcs_problem* pb, const double* b, double* x, mcs_solve_info* info, double* red,
                         double* scal, double* host, double* host_dev) {
  int rc = MCS_OK;
  hipStream_t st = pb->stream;
  const int64_t n = pb->ndof;
  mcs_solve_info inf{};
  auto t0 = std::chrono::steady_clock::now();
  Ctx<double> c64(pb);
  c64.host_dev = host_dev;
  c64.red = red;
  c64.scal = scal;
  if (pb->opt.precision == 0) {
    int its = 0;
    double rel = 0, b1 = 0;
    rc = c64.minres(b, x, pb->opt.tol, pb->opt.max_it, -1.0, -1.0, &its, &rel, &b1, host);
    inf.iterations = its;
    inf.outer_steps = 1;
    inf.rel_precond_residual = rel;
  } else {
    Ctx<float> c32(pb);
    c32.host_dev = host_dev;
    c32.red = red;
    c32.scal = scal;
    double* r64 = c64.v(VR64);
    float* r32 = c32.v(VB64);   // slot beyond the FP32 MINRES vectors
    float* d32 = c32.v(VX64);
    launch_fill<double>(st, n, 0.0, x);
    launch_axpby<double>(st, n, 1.0, b, 0.0, r64);
    double beta0 = -1.0, rel = 1.0;
    int total = 0, outer = 0;
    rc = MCS_OK;
    for (outer = 0; outer < pb->opt.max_outer; ++outer) {
      double rn = std::sqrt(c64.dot(r64, r64, host));
      if (!std::isfinite(rn)) {
        rc = MCS_ERR_NONFINITE;
        break;
      }
      if (rn == 0.0) {
        rel = 0.0;
        break;
      }
      launch_scale_convert<double, float>(st, n, 1.0 / rn, r64, r32, 0);
      int its = 0;
      double irel = 0, b1 = 0;
      // skip when the outer residual is already small enough; otherwise reduce
      // by inner_tol, or only as far as the outer target needs (with margin 4)
      double stop = (beta0 > 0) ? pb->opt.tol * beta0 / rn : -1.0;
      double abs_stop = (beta0 > 0) ? 0.25 * pb->opt.tol * beta0 / rn : -1.0;
      int irc = c32.minres(r32, d32, pb->opt.inner_tol, pb->opt.max_it, stop, abs_stop, &its, &irel, &b1, host);
      if (beta0 < 0) beta0 = b1 * rn;
      rel = b1 * rn / beta0;
      total += its;
      if (irc == MCS_ERR_NONFINITE || irc == MCS_ERR_BREAKDOWN) {
        rc = irc;
        break;
      }
      if (rel <= pb->opt.tol) break;   // current outer residual already small enough
      launch_scale_convert<float, double>(st, n, rn, d32, x, 1);
      // r = b - K x in FP64
      double* kx = c64.v(VT64);
      c64.apply(x, kx, 1 | 2 | 4);
      launch_axpby<double>(st, n, 1.0, b, 0.0, r64);
      launch_axpby<double>(st, n, -1.0, kx, 1.0, r64);
    }
    if (rc == MCS_OK && rel > pb->opt.tol) rc = MCS_ERR_NOT_CONVERGED;
    inf.iterations = total;
    inf.outer_steps = outer + 1;
    inf.rel_precond_residual = rel;
  }
  HIPCHK(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  inf.t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  // true residual ||b - K x|| / ||b|| in FP64 (before pressure normalisation;
  // the constant pressure mode is in the kernel of K)
  {
    double* kx = c64.v(VT64);
    double* rr = c64.v(VR64);
    c64.apply(x, kx, 1 | 2 | 4);
    launch_axpby<double>(st, n, 1.0, b, 0.0, rr);
    launch_axpby<double>(st, n, -1.0, kx, 1.0, rr);
    double rn = c64.dot(rr, rr, host);
    double bn = c64.dot(b, b, host);
    inf.rel_residual = bn > 0 ? std::sqrt(rn / bn) : std::sqrt(rn);
  }
  SolveParams P = solve_params(pb);
  if (!pb->has_outlet) launch_pressure_mean(st, P, pb->p.rpmom, pb->p.rpconst, x, red);
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    set_error("HIP error '%s' in solve", hipGetErrorString(he));
    return MCS_ERR_HIP;
  }
  inf.status = rc;
  if (info) *info = inf;
  if (rc) set_error("solve: %s after %d iterations (rel %.3e)", mcs_status_string(rc), inf.iterations,
                    inf.rel_precond_residual);
  return rc;
}


int mcs_solve_rhs(mcs_problem* pb, const double* b, double* x, mcs_solve_info* info) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_solve needs mcs_condense first");
    return MCS_ERR_STATE;
  }
  if (!b || !x) {
    set_error("null vector");
    return MCS_ERR_ARG;
  }
  // pinned scalars of the host-side recurrences, released on every return path
  struct Pinned {
    double* p = nullptr;
    ~Pinned() {
      ApiLock lock(device_api_mutex());
      if (p) hipHostFree(p);
    }
  } pin;
  {
    ApiLock lock(device_api_mutex());
    HIPCHK(hipHostMalloc((void**)&pin.p, 64));
  }
  double* host_dev = nullptr;
  HIPCHK(hipHostGetDevicePointer((void**)&host_dev, pin.p, 0));
  return solve_rhs_run(pb, b, x, info, pb->p.red, pb->p.scal, pin.p, host_dev);
}

int mcs_solve_rhs_noalloc(mcs_problem* pb, const double* b, double* x, mcs_solve_info* info) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_solve_rhs_noalloc needs mcs_condense first");
    return MCS_ERR_STATE;
  }
  if (!b || !x) {
    set_error("null vector");
    return MCS_ERR_ARG;
  }
  double* sp = (pb->device >= 0 && pb->device < NOALLOC_MAX_DEVICES) ? noalloc_scratch_ptr[pb->device] : nullptr;
  if (!sp) {
    set_error("mcs_solve_rhs_noalloc: no scratch address for device %d (bind the problem first)", pb->device);
    return MCS_ERR_STATE;
  }
  // partial sums of a dot product (one per reduction block) and the scalar
  // slot behind them; every kernel writes its slots before reading them
  const int64_t parts = std::min<int64_t>(1024, std::max<int64_t>(1, (pb->ndof + 255) / 256));
  if (parts + 1 > NOALLOC_SCRATCH_DOUBLES) {
    set_error("mcs_solve_rhs_noalloc: %lld reduction slots exceed the scratch of %lld doubles", (long long)(parts + 1),
              (long long)NOALLOC_SCRATCH_DOUBLES);
    return MCS_ERR_WORKSPACE;
  }
  double host[2] = {0.0, 0.0};
  return solve_rhs_run(pb, b, x, info, sp, sp + 1024, host, nullptr);
}

int mcs_solve(mcs_problem* pb, const double* f_lattice, double* x, mcs_solve_info* info) {
  int rc = check_bound(pb);
  if (rc) return rc;
  double* b = Ctx<double>(pb).v(VB64);
  rc = mcs_load(pb, f_lattice, b);
  if (rc) return rc;
  return mcs_solve_rhs(pb, b, x, info);
}

int mcs_get_array(mcs_problem* pb, const char* name, void** ptr, int64_t* count) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!name || !ptr || !count) {
    set_error("null argument");
    return MCS_ERR_ARG;
  }
  const Sizes& s = pb->sz;
  struct E {
    const char* n;
    int64_t cnt;
  } table[] = {{"Ad", pb->ne * s.nd * s.nd},   {"H", pb->ne * s.nb * s.nd},
               {"Aoo", pb->ne * s.nb * s.nb},  {"Aooinv", pb->ne * s.nb * s.nb},  {"Dinv", pb->nff * s.nfb * s.nfb},
               {"EF", pb->nff * s.nfb * pb->d * pb->d}, {"Ad32", pb->ne * s.nd * s.nd}, {"H32", pb->ne * s.nb * s.nd},
               {"detJ", pb->ne},               {"colour_desc", pb->nff * 4},        {"elem_ff", pb->ne * (pb->d + 1)},
               {"W", pb->ne * (pb->d + 1) * pb->d * s.nd}, {"Cinv", pb->ncinv},
               {"mgA0", pb->mg[0].nvert * (pb->d == 3 ? 27 : 9) * pb->d * pb->d}};
  for (auto& e : table)
    if (!strcmp(e.n, name)) {
      *ptr = ws_ptr<char>(pb, name);
      *count = e.cnt;
      if (!*ptr) {
        set_error("array '%s' is not stored in this layout", name);
        return MCS_ERR_STATE;
      }
      return MCS_OK;
    }
  set_error("unknown array '%s'", name);
  return MCS_ERR_ARG;
}

int mcs_get_full_colouring(const mcs_problem* pb, int64_t* n_blocks, int32_t* colour_host) {
  if (!pb || !n_blocks) {
    set_error("null argument");
    return MCS_ERR_ARG;
  }
  *n_blocks = pb->nblk;
  if (colour_host) std::copy(pb->h_blk_colour.begin(), pb->h_blk_colour.end(), colour_host);
  return MCS_OK;
}

int mcs_get_topology(const mcs_problem* pb, int32_t* colour_host, int32_t* elem_ff_host) {
  if (!pb) {
    set_error("null problem");
    return MCS_ERR_ARG;
  }
  if (colour_host) std::copy(pb->h_colour.begin(), pb->h_colour.end(), colour_host);
  if (elem_ff_host) std::copy(pb->h_elem_ff.begin(), pb->h_elem_ff.end(), elem_ff_host);
  return MCS_OK;
}

int mcs_timer_enable(mcs_problem* pb, int enable) {
  int rc = check_bound(pb);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(pb->stream));
  timer_flush(pb);
  if (enable < 0) {
    set_error("mcs_timer_enable: enable must be 0 (off) or a sampling period >= 1");
    return MCS_ERR_ARG;
  }
  pb->timer_on = enable != 0;
  pb->timer_period = enable > 0 ? enable : 1;
  pb->t_tick[0] = pb->t_tick[1] = 0;
  for (int i = 0; i < 2; ++i) {
    pb->t_ms[i] = 0.0;
    pb->t_bytes[i] = 0.0;
    pb->t_launches[i] = 0;
  }
  HIPCHK(hipMemsetAsync(work_counters(pb), 0, WCOUNT * sizeof(unsigned long long), pb->stream));
  HIPCHK(hipStreamSynchronize(pb->stream));
  return MCS_OK;
}

int mcs_timer_read(mcs_problem* pb, int32_t kernel, double* total_ms, int64_t* launches, double* bytes) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (kernel != MCS_TIMER_SMOOTH && kernel != MCS_TIMER_KAPPLY) {
    set_error("mcs_timer_read: kernel must be MCS_TIMER_SMOOTH or MCS_TIMER_KAPPLY");
    return MCS_ERR_ARG;
  }
  HIPCHK(hipStreamSynchronize(pb->stream));
  timer_flush(pb);
  std::vector<unsigned long long> wc(WCOUNT);
  HIPCHK(hipMemcpyAsync(wc.data(), work_counters(pb), WCOUNT * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         pb->stream));
  HIPCHK(hipStreamSynchronize(pb->stream));
  unsigned long long cnt[2] = {0, 0};
  for (int i = 0; i < 256; ++i) {
    cnt[0] += wc[i * 16];
    cnt[1] += wc[256 * 16 + i * 16];
  }
  // smoother bytes: counted on the device for the condensed sweeps, on the
  // host (per colour phase) for the full-system sweeps
  const double smooth_bytes =
      pb->t_bytes[0] + cnt[0] * smooth_bytes_per_facet(pb->sz, 8) + cnt[1] * smooth_bytes_per_facet(pb->sz, 4);
  if (total_ms) *total_ms = pb->t_ms[kernel];
  if (launches) *launches = pb->t_launches[kernel];
  if (bytes) *bytes = kernel == MCS_TIMER_SMOOTH ? smooth_bytes : pb->t_bytes[kernel];
  return MCS_OK;
}

int mcs_eval(mcs_problem* pb, const double* x, int32_t n_pts, const double* ref_pts_host, double* u_vals,
             double* p_vals) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {  // the Piola factors use det J from the condensation
    set_error("mcs_eval: call mcs_condense first");
    return MCS_ERR_STATE;
  }
  const int nv = pb->d + 1;
  if (!x || !ref_pts_host || !u_vals || !p_vals || n_pts <= 0 || (int64_t)n_pts * nv > pb->nred) {
    set_error("mcs_eval: null pointer or n_pts outside 1..%lld", (long long)(pb->nred / nv));
    return MCS_ERR_ARG;
  }
  HIPCHK(hipMemcpyAsync(pb->p.red, ref_pts_host, (size_t)n_pts * nv * 8, hipMemcpyHostToDevice, pb->stream));
  SolveParams P = solve_params(pb);
  if (pb->has_dirichlet) P.xD = pb->p.xD;
  launch_eval(pb->stream, P, pb->p.coords, pb->p.elem_verts, pb->p.elem_perm, pb->p.rphi, pb->p.rpidx, n_pts,
              pb->p.red, x, u_vals, p_vals);
  HIPCHK(hipStreamSynchronize(pb->stream));
  return MCS_OK;
}

int mcs_eval_stress(mcs_problem* pb, const double* x, int32_t n_pts, const double* ref_pts_host,
                    double* sigma_vals, double* omega_vals) {
  int rc = check_bound(pb);
  if (rc) return rc;
  if (!pb->condensed) {
    set_error("mcs_eval_stress: call mcs_condense first");
    return MCS_ERR_STATE;
  }
  const int nv = pb->d + 1;
  if (!x || !ref_pts_host || !sigma_vals || !omega_vals || n_pts <= 0 || (int64_t)n_pts * nv > pb->nred) {
    set_error("mcs_eval_stress: null pointer or n_pts outside 1..%lld", (long long)(pb->nred / nv));
    return MCS_ERR_ARG;
  }
  hipStream_t st = pb->stream;
  int* status = reinterpret_cast<int*>(pb->p.scal + 200);
  HIPCHK(hipMemsetAsync(status, 0, sizeof(int), st));
  HIPCHK(hipMemcpyAsync(pb->p.red, ref_pts_host, (size_t)n_pts * nv * 8, hipMemcpyHostToDevice, st));
  StressParams S{};
  S.C = cond_params(pb, status);
  S.x = x;
  S.elem_ff = pb->p.elem_ff;
  S.elem_perm = pb->p.elem_perm;
  S.off_f = pb->off_f;
  S.xD = pb->has_dirichlet ? pb->p.xD : nullptr;
  S.rpsi = pb->p.rpsi;
  S.rpsib = pb->p.rpsib;
  S.npts = n_pts;
  S.pts = pb->p.red;
  S.sig = sigma_vals;
  S.om = omega_vals;
  launch_stress(st, S, (int)pb->n_slots);
  return sync_status(pb, "mcs_eval_stress");
}

int mcs_get_launch_config(const mcs_problem* pb, int dt, int32_t* facets_per_block, int64_t* grid_cap, double* us) {
  if (!pb || (dt != MCS_F64 && dt != MCS_F32)) {
    set_error("launch config: bad argument");
    return MCS_ERR_ARG;
  }
  const int slot = dt == MCS_F64 ? 0 : 1;
  if (facets_per_block) *facets_per_block = pb->tune_fpw[slot];
  if (grid_cap) *grid_cap = pb->tune_cap[slot];
  if (us) *us = pb->tune_us[slot];
  return MCS_OK;
}

int mcs_set_launch_config(mcs_problem* pb, int dt, int32_t facets_per_block, int64_t grid_cap) {
  if (!pb || (dt != MCS_F64 && dt != MCS_F32) || (facets_per_block != 1 && facets_per_block != 2) || grid_cap < 0) {
    set_error("launch config: bad argument");
    return MCS_ERR_ARG;
  }
  if (dt == MCS_F64 && pb->lean) {
    set_error("launch config: precision 1 has no FP64 smoother");
    return MCS_ERR_ARG;
  }
  const int slot = dt == MCS_F64 ? 0 : 1;
  pb->tune_fpw[slot] = facets_per_block;
  pb->tune_cap[slot] = grid_cap;
  pb->tune_us[slot] = 0.0;
  pb->tune_fixed[slot] = true;
  return MCS_OK;
}

int mcs_get_apply_config(const mcs_problem* pb, int dt, int32_t* rows_per_thread, double* us) {
  if (!pb || (dt != MCS_F64 && dt != MCS_F32)) {
    set_error("apply config: bad argument");
    return MCS_ERR_ARG;
  }
  const int slot = dt == MCS_F64 ? 0 : 1;
  if (rows_per_thread) *rows_per_thread = pb->tune_rpt[slot];
  if (us) *us = pb->tune_rpt_us[slot];
  return MCS_OK;
}

int mcs_set_apply_config(mcs_problem* pb, int dt, int32_t rows_per_thread) {
  if (!pb || (dt != MCS_F64 && dt != MCS_F32) ||
      !(rows_per_thread == 0 || rows_per_thread == 1 || rows_per_thread == 2 ||
        (rows_per_thread == 4 && dt == MCS_F32))) {
    set_error("apply config: dt must be MCS_F64 or MCS_F32 and rows_per_thread 0, 1, 2 (or 4 in FP32)");
    return MCS_ERR_ARG;
  }
  const int slot = dt == MCS_F64 ? 0 : 1;
  pb->tune_rpt[slot] = rows_per_thread;
  pb->tune_rpt_us[slot] = 0.0;
  pb->tune_rpt_fixed[slot] = true;
  return MCS_OK;
}

int mcs_set_solve_options(mcs_problem* pb, double tol, int32_t max_it, double inner_tol, int32_t max_outer) {
  if (!pb || !std::isfinite(tol) || tol < 0.0 || max_it < 1 || !std::isfinite(inner_tol) || inner_tol < 0.0 ||
      inner_tol >= 1.0 || max_outer < 1) {
    set_error("solve options: bad argument");
    return MCS_ERR_ARG;
  }
  pb->opt.tol = tol;
  pb->opt.max_it = max_it;
  pb->opt.inner_tol = inner_tol;
  pb->opt.max_outer = max_outer;
  return MCS_OK;
}

void mcs_destroy(mcs_problem* pb) {
  ApiLock lock(device_api_mutex());
  delete pb;
}

}  // extern "C"
