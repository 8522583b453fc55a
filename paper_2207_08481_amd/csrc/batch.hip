// Batched solves of many independent MCS Stokes problems.
//
// Members with the same dimension and order are merged into one union
// (plan_union): every element, facet and lattice kernel of the single-problem
// path then runs once per group over all members.  Preconditioned MINRES
// (Paige-Saunders) runs per member with its scalars in device memory
// (kernels_batch.hip); members whose iteration has ended are masked out of
// every kernel, and the iterations of all groups (one HIP stream each) are
// captured once as a graph and replayed.  Precision 1 refines every member in
// FP64 on its own true residual, as mcs_solve does for one problem.
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <utility>

#include "ctx.h"

namespace mcs {
int plan_problem(const mcs_mesh* mesh, const mcs_options* opt, mcs_problem* pb);
int plan_union(const std::vector<const mcs_problem*>& parts, mcs_problem* u);
int layout_workspace(mcs_problem* pb);
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

namespace {

constexpr int64_t TILE = 4096;   // dofs per reduction / update tile

struct Group {
  std::unique_ptr<mcs_problem> u;
  std::vector<int> members;        // batch indices, in union order
  std::vector<SegTile> h_tiles;
  std::vector<int32_t> h_tile_off, h_elem_prob, h_facet_prob;
  std::vector<int64_t> h_pe0;
  size_t off_u = 0, off_arr = 0, arr_bytes = 0;
  int64_t fun_doubles = 0;
  // device arrays (inside the batch workspace)
  SegTile* tiles = nullptr;
  int32_t* tile_off = nullptr;
  double* partial = nullptr;
  double* st = nullptr;
  int32_t *act = nullptr, *go = nullptr, *its = nullptr, *status = nullptr, *done = nullptr;
  int32_t *elem_prob = nullptr, *facet_prob = nullptr;
  int64_t* pe0 = nullptr;
  double* fun = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_join = nullptr;
  // pinned host mirrors: st, then its / status / act
  double* h_st = nullptr;
  int32_t* h_int = nullptr;

  int np() const { return (int)members.size(); }
  SegDev seg(int32_t* mask, int maxit) const {
    SegDev S{};
    S.nprob = np();
    S.ntiles = (int64_t)h_tiles.size();
    S.tiles = tiles;
    S.tile_off = tile_off;
    S.partial = partial;
    S.st = st;
    S.active = mask;
    S.its = its;
    S.status = status;
    S.done = done;
    S.maxit = maxit;
    return S;
  }
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void fill_info(const mcs_problem* pb, mcs_info* info) {
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
  info->n_mg_levels = (int32_t)pb->plev[0].size();
  info->workspace_bytes = 0;
}

}  // namespace

struct mcs_batch {
  int n = 0;
  mcs_options opt{};
  std::vector<std::unique_ptr<mcs_problem>> singles;
  std::vector<Group> groups;
  std::vector<int> grp, idx;        // member -> group, position in the group
  size_t ws_bytes = 0;
  void* ws = nullptr;
  hipStream_t user = nullptr, main = nullptr;
  hipEvent_t ev_fork = nullptr;
  int device = -1;
  bool condensed = false;
  int use_graph = 1, chunk = 6;
  bool timer = false;               // smoother timing: launches one by one
  hipGraphExec_t gexec[2] = {nullptr, nullptr};   // inner iteration chunk, FP64 / FP32
  // mcs_batch_solve_async: 0 no solve started, 1 running, 2 finished and not
  // yet collected by mcs_batch_wait
  std::atomic<int> async_state{0};
  std::thread async_thread;
  std::vector<const double*> async_f;
  std::vector<double*> async_x;
  std::vector<mcs_solve_info> async_inf;
  int async_rc = 0;
  std::string async_err;
  ~mcs_batch() {
    for (auto& g : gexec)
      if (g) hipGraphExecDestroy(g);
    for (auto& G : groups) {
      if (G.ev_join) hipEventDestroy(G.ev_join);
      if (G.stream) hipStreamDestroy(G.stream);
      if (G.h_st) hipHostFree(G.h_st);
      if (G.h_int) hipHostFree(G.h_int);
    }
    if (ev_fork) hipEventDestroy(ev_fork);
    if (main) hipStreamDestroy(main);
  }
};

namespace {

// Calls other than poll, wait and destroy are refused while an asynchronous
// solve has not been collected.
bool async_busy(const mcs_batch* B) {
  if (B && B->async_state.load(std::memory_order_acquire) != 0) {
    set_error("an asynchronous solve of this batch is in flight (mcs_batch_wait collects it)");
    return true;
  }
  return false;
}

// main stream -> every group stream
int fork(mcs_batch* B) {
  HIPCHK(hipEventRecord(B->ev_fork, B->main));
  for (auto& G : B->groups) HIPCHK(hipStreamWaitEvent(G.stream, B->ev_fork, 0));
  return MCS_OK;
}
// every group stream -> main stream
int join(mcs_batch* B) {
  for (auto& G : B->groups) {
    HIPCHK(hipEventRecord(G.ev_join, G.stream));
    HIPCHK(hipStreamWaitEvent(B->main, G.ev_join, 0));
  }
  return MCS_OK;
}

// Per-group MINRES state for work precision R.  The vectors live in the
// union's work slots; r1, r2, kv rotate with period 3 and w1, w2 with period 2,
// so a run of 6 iterations returns every pointer to its role.
template <typename R>
struct GroupRun {
  Group* G;
  Ctx<R> c;
  SegDev S;
  R *x, *r1, *r2, *y, *vv, *w1, *w2, *kv;
  GroupRun(Group* g, int maxit, R* xout) : G(g), c(g->u.get()) {
    c.set_mask(g->elem_prob, g->facet_prob, g->act);
    S = g->seg(g->act, maxit);
    x = xout;
    r1 = c.v(VR1);
    r2 = c.v(VR2);
    y = c.v(VY);
    vv = c.v(VV);
    w1 = c.v(VW1);
    w2 = c.v(VW2);
    kv = c.v(VKV);
  }
  // x = 0, r2 = b, y = K-hat^{-1} r2, beta1 and the entry test (k_mr_init)
  void start(const R* b) {
    hipStream_t st = c.st;
    const int64_t n = c.n;
    launch_fill<R>(st, n, R(0), x);
    launch_fill<R>(st, n, R(0), r1);
    launch_fill<R>(st, n, R(0), w1);
    launch_fill<R>(st, n, R(0), w2);
    launch_axpby<R>(st, n, 1.0, b, 0.0, r2);
    c.khat(r2, y);
    launch_seg_dot<R>(st, S, r2, y, ST_BB);
    launch_mr_init(st, S);
  }
  void iteration() {
    hipStream_t st = c.st;
    launch_seg_scale<R>(st, S, y, vv, ST_BETA, 1);          // v = y / beta
    c.apply(vv, kv, 1 | 2 | 4);                              // K v
    launch_seg_axpy_ratio<R>(st, S, r1, kv, ST_BETA, ST_OLDB, 1);
    launch_seg_dot<R>(st, S, vv, kv, ST_ALPHA);
    launch_seg_axpy_ratio<R>(st, S, r2, kv, ST_ALPHA, ST_BETA, 0);
    R* t = r1;
    r1 = r2;
    r2 = kv;
    kv = t;
    c.khat(r2, y);
    launch_seg_dot<R>(st, S, r2, y, ST_BB);
    launch_mr_update(st, S);
    launch_seg_w<R>(st, S, vv, w1, w2, x);
    launch_mr_retire(st, S);
    std::swap(w1, w2);
  }
};

// Copies every group's mask `which` (0: act, 1: go) to the host and returns
// whether any member is set.  Synchronises the main stream.
int any_set(mcs_batch* B, int which, bool* any) {
  for (auto& G : B->groups)
    HIPCHK(hipMemcpyAsync(G.h_int + 2 * G.np(), which ? G.go : G.act, G.np() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, B->main));
  HIPCHK(hipStreamSynchronize(B->main));
  *any = false;
  for (auto& G : B->groups)
    for (int j = 0; j < G.np(); ++j)
      if (G.h_int[2 * G.np() + j]) *any = true;
  return MCS_OK;
}

// Runs the MINRES iterations of all groups (already started) until every
// member has left: chunks of B->chunk iterations, replayed from a captured
// graph or launched one by one.
template <typename R>
int run_iterations(mcs_batch* B, std::vector<GroupRun<R>>& runs, int maxit) {
  const int prec = sizeof(R) == 8 ? 0 : 1;
  // With the kernel timer on, the groups run one after another so that each
  // timed launch has the device to itself.
  auto enqueue_chunk = [&]() -> int {
    int rc = fork(B);
    if (rc) return rc;
    for (size_t g = 0; g < runs.size(); ++g) {
      if (B->timer && g > 0) {
        HIPCHK(hipEventRecord(runs[g - 1].G->ev_join, runs[g - 1].G->stream));
        HIPCHK(hipStreamWaitEvent(runs[g].G->stream, runs[g - 1].G->ev_join, 0));
      }
      for (int i = 0; i < B->chunk; ++i) runs[g].iteration();
    }
    return join(B);
  };
  if (B->use_graph && !B->timer && !B->gexec[prec]) {
    ApiLock lock(device_api_mutex());
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(B->main, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_chunk();
    hipError_t e = hipStreamEndCapture(B->main, &graph);
    if (rc) return rc;
    HIPCHK(e);
    e = hipGraphInstantiate(&B->gexec[prec], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    HIPCHK(e);
  }
  const bool graph = B->use_graph && !B->timer;
  const int max_chunks = maxit / B->chunk + 2;
  for (int k = 0; k < max_chunks; ++k) {
    bool any = false;
    int rc = any_set(B, 0, &any);
    if (rc) return rc;
    if (!any) return MCS_OK;
    if (graph) {
      HIPCHK(hipGraphLaunch(B->gexec[prec], B->main));
    } else {
      rc = enqueue_chunk();
      if (rc) return rc;
    }
  }
  set_error("batched MINRES did not terminate");
  return MCS_ERR_STATE;
}

int upload_fields(Group& G, std::initializer_list<int> fields) {
  const int np = G.np();
  for (int f : fields)
    HIPCHK(hipMemcpyAsync(G.st + (size_t)f * np, G.h_st + (size_t)f * np, np * sizeof(double), hipMemcpyHostToDevice,
                          G.stream));
  return MCS_OK;
}

}  // namespace

extern "C" {

int mcs_batch_plan(const mcs_mesh* meshes, const int32_t* orders, int32_t n, const mcs_options* options,
                   mcs_batch** out, mcs_batch_info* info) {
  if (!meshes || !orders || !options || !out || n <= 0) {
    set_error("batch plan: null argument or empty batch");
    return MCS_ERR_ARG;
  }
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 6; ++a)
      if (meshes[i].face_bc[a] != 0) {
        set_error("batch plan: member %d has an outlet face; batches take all-Dirichlet problems", i);
        return MCS_ERR_UNSUPPORTED;
      }
  if (options->smoother == 2) {
    set_error("batch plan: the full-system variant (smoother 2) is for single problems");
    return MCS_ERR_UNSUPPORTED;
  }
  *out = nullptr;
  std::unique_ptr<mcs_batch> B(new (std::nothrow) mcs_batch());
  if (!B) {
    set_error("out of host memory");
    return MCS_ERR_ARG;
  }
  B->n = n;
  B->opt = *options;
  B->grp.assign(n, -1);
  B->idx.assign(n, -1);
  std::map<std::pair<int, int>, int> gid;
  try {
    for (int i = 0; i < n; ++i) {
      mcs_options o = *options;
      o.order = orders[i];
      B->singles.emplace_back(new mcs_problem());
      int rc = plan_problem(&meshes[i], &o, B->singles.back().get());
      if (rc) {
        std::string msg = last_error();
        set_error("member %d: %s", i, msg.c_str());
        return rc;
      }
      auto key = std::make_pair(meshes[i].dim, orders[i]);
      auto it = gid.find(key);
      if (it == gid.end()) {
        it = gid.emplace(key, (int)B->groups.size()).first;
        B->groups.emplace_back();
      }
      Group& G = B->groups[it->second];
      B->grp[i] = it->second;
      B->idx[i] = (int)G.members.size();
      G.members.push_back(i);
    }
    B->opt = B->singles[0]->opt;   // defaults filled in by the planner
    B->opt.order = 0;
    size_t off = 0;
    for (auto& G : B->groups) {
      std::vector<const mcs_problem*> parts;
      for (int i : G.members) parts.push_back(B->singles[i].get());
      G.u.reset(new mcs_problem());
      int rc = plan_union(parts, G.u.get());
      if (rc) return rc;
      mcs_problem* u = G.u.get();
      u->ref = build_ref_tables(u->d, u->sz.k);
      rc = layout_workspace(u);
      if (rc) return rc;
      const Sizes& s = u->sz;
      const int np = G.np();
      // tiles: per member its bubble, facet and pressure sections
      G.h_tile_off.assign(1, 0);
      for (int j = 0; j < np; ++j) {
        const int64_t sec[3][2] = {{u->pe0[j] * s.nb, u->pe0[j + 1] * s.nb},
                                   {u->off_f + u->pf0[j] * s.nfb, u->off_f + u->pf0[j + 1] * s.nfb},
                                   {u->off_p + u->pe0[j] * s.np, u->off_p + u->pe0[j + 1] * s.np}};
        for (auto& r : sec)
          for (int64_t a = r[0]; a < r[1]; a += TILE) G.h_tiles.push_back({j, (int32_t)std::min(TILE, r[1] - a), a});
        G.h_tile_off.push_back((int32_t)G.h_tiles.size());
      }
      G.h_elem_prob.resize(u->ne);
      G.h_facet_prob.resize(u->nff);
      for (int j = 0; j < np; ++j) {
        for (int64_t e = u->pe0[j]; e < u->pe0[j + 1]; ++e) G.h_elem_prob[e] = j;
        for (int64_t g = u->pf0[j]; g < u->pf0[j + 1]; ++g) G.h_facet_prob[g] = j;
      }
      G.h_pe0 = u->pe0;
      G.fun_doubles = u->ne * (int64_t)s.nlat * u->d;
      // group arrays after the union workspace
      G.off_u = off;
      off = align_up(off + u->ws_bytes, 4096);
      G.off_arr = off;
      const int64_t nt = (int64_t)G.h_tiles.size();
      size_t a = 0;
      auto add = [&](size_t bytes) {
        a = align_up(a, 256);
        size_t r = a;
        a += bytes;
        return r;
      };
      size_t o_tiles = add(nt * sizeof(SegTile)), o_toff = add((np + 1) * 4), o_part = add(nt * 8),
             o_st = add((size_t)ST_NFIELD * np * 8), o_act = add(np * 4), o_go = add(np * 4), o_its = add(np * 4),
             o_status = add(np * 4), o_done = add(np * 4), o_ep = add(u->ne * 4), o_fp = add(u->nff * 4),
             o_pe0 = add((np + 1) * 8), o_fun = add(G.fun_doubles * 8);
      G.arr_bytes = align_up(a, 4096);
      off += G.arr_bytes;
      // remember the relative offsets through the pointers (rebased at bind)
      G.tiles = reinterpret_cast<SegTile*>(o_tiles);
      G.tile_off = reinterpret_cast<int32_t*>(o_toff);
      G.partial = reinterpret_cast<double*>(o_part);
      G.st = reinterpret_cast<double*>(o_st);
      G.act = reinterpret_cast<int32_t*>(o_act);
      G.go = reinterpret_cast<int32_t*>(o_go);
      G.its = reinterpret_cast<int32_t*>(o_its);
      G.status = reinterpret_cast<int32_t*>(o_status);
      G.done = reinterpret_cast<int32_t*>(o_done);
      G.elem_prob = reinterpret_cast<int32_t*>(o_ep);
      G.facet_prob = reinterpret_cast<int32_t*>(o_fp);
      G.pe0 = reinterpret_cast<int64_t*>(o_pe0);
      G.fun = reinterpret_cast<double*>(o_fun);
    }
    B->ws_bytes = off;
  } catch (const std::exception& ex) {
    set_error("batch plan failed: %s", ex.what());
    return MCS_ERR_ARG;
  }
  if (info) {
    info->n_problems = n;
    info->n_groups = (int32_t)B->groups.size();
    int64_t tot = 0;
    for (auto& p : B->singles) tot += p->ndof;
    info->n_dof_total = tot;
    info->workspace_bytes = B->ws_bytes;
  }
  *out = B.release();
  return MCS_OK;
}

int mcs_batch_member_info(const mcs_batch* B, int32_t i, mcs_info* info) {
  if (!B || !info || i < 0 || i >= B->n) {
    set_error("batch member info: bad argument");
    return MCS_ERR_ARG;
  }
  fill_info(B->singles[i].get(), info);
  return MCS_OK;
}

int mcs_batch_set_mode(mcs_batch* B, int use_graph, int chunk) {
  if (async_busy(B)) return MCS_ERR_STATE;
  if (!B || chunk <= 0 || chunk % 6 != 0) {
    set_error("batch mode: chunk must be a positive multiple of 6");
    return MCS_ERR_ARG;
  }
  ApiLock lock(device_api_mutex());
  if (chunk != B->chunk)
    for (auto& g : B->gexec)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
  B->use_graph = use_graph ? 1 : 0;
  B->chunk = chunk;
  return MCS_OK;
}

int mcs_batch_bind(mcs_batch* B, void* workspace, size_t bytes, void* stream) {
  if (async_busy(B)) return MCS_ERR_STATE;
  ApiLock lock(device_api_mutex());
  if (!B) {
    set_error("null batch");
    return MCS_ERR_ARG;
  }
  if (!workspace || bytes < B->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
    set_error("batch workspace must be >= %zu bytes and 256-byte aligned", B->ws_bytes);
    return MCS_ERR_WORKSPACE;
  }
  if (B->ws) {
    set_error("batch is already bound");
    return MCS_ERR_STATE;
  }
  HIPCHK(hipGetDevice(&B->device));
  B->ws = workspace;
  B->user = static_cast<hipStream_t>(stream);
  HIPCHK(hipStreamCreateWithFlags(&B->main, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
  char* base = static_cast<char*>(workspace);
  for (auto& G : B->groups) {
    HIPCHK(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&G.ev_join, hipEventDisableTiming));
    int rc = mcs_bind(G.u.get(), base + G.off_u, G.u->ws_bytes, G.stream);
    if (rc) return rc;
    char* ab = base + G.off_arr;
    auto rebase = [&](auto*& p) { p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(ab + reinterpret_cast<size_t>(p)); };
    rebase(G.tiles);
    rebase(G.tile_off);
    rebase(G.partial);
    rebase(G.st);
    rebase(G.act);
    rebase(G.go);
    rebase(G.its);
    rebase(G.status);
    rebase(G.done);
    rebase(G.elem_prob);
    rebase(G.facet_prob);
    rebase(G.pe0);
    rebase(G.fun);
    const int np = G.np();
    HIPCHK(hipHostMalloc((void**)&G.h_st, (size_t)ST_NFIELD * np * sizeof(double)));
    HIPCHK(hipHostMalloc((void**)&G.h_int, (size_t)4 * np * sizeof(int32_t)));
    std::memset(G.h_st, 0, (size_t)ST_NFIELD * np * sizeof(double));
    hipStream_t st = G.stream;
    HIPCHK(hipMemsetAsync(ab, 0, G.arr_bytes, st));
    HIPCHK(hipMemcpyAsync(G.tiles, G.h_tiles.data(), G.h_tiles.size() * sizeof(SegTile), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.tile_off, G.h_tile_off.data(), G.h_tile_off.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.elem_prob, G.h_elem_prob.data(), G.h_elem_prob.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.facet_prob, G.h_facet_prob.data(), G.h_facet_prob.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.pe0, G.h_pe0.data(), G.h_pe0.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.st, G.h_st, (size_t)ST_NFIELD * np * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return MCS_OK;
}

int mcs_batch_condense(mcs_batch* B, const double* const* nu) {
  if (async_busy(B)) return MCS_ERR_STATE;
  if (!B || !B->ws) {
    set_error("batch is not bound");
    return B ? MCS_ERR_STATE : MCS_ERR_ARG;
  }
  if (!nu) {
    set_error("null viscosity array");
    return MCS_ERR_ARG;
  }
  if (B->user) HIPCHK(hipStreamSynchronize(B->user));
  for (auto& G : B->groups) {
    mcs_problem* u = G.u.get();
    // member viscosities, in union order, staged in the element scratch
    double* stage = u->p.escr;
    for (int j = 0; j < G.np(); ++j) {
      const int m = G.members[j];
      if (!nu[m]) {
        set_error("member %d: null viscosity", m);
        return MCS_ERR_ARG;
      }
      HIPCHK(hipMemcpyAsync(stage + u->pe0[j], nu[m], (u->pe0[j + 1] - u->pe0[j]) * sizeof(double),
                            hipMemcpyDeviceToDevice, G.stream));
    }
    int rc = mcs_condense(u, stage);
    if (rc) return rc;
  }
  B->condensed = true;
  return MCS_OK;
}

}  // extern "C"

namespace {

// The body of mcs_batch_solve (also run on the thread of mcs_batch_solve_async).
int batch_solve(mcs_batch* B, const double* const* f, double* const* xo, mcs_solve_info* infos) {
  if (!B || !B->ws || !B->condensed) {
    set_error("batch solve needs bind and condense first");
    return B ? MCS_ERR_STATE : MCS_ERR_ARG;
  }
  if (!f || !xo) {
    set_error("null force or solution array");
    return MCS_ERR_ARG;
  }
  for (int i = 0; i < B->n; ++i)
    if (!f[i] || !xo[i]) {
      set_error("member %d: null force or solution pointer", i);
      return MCS_ERR_ARG;
    }
  if (B->user) HIPCHK(hipStreamSynchronize(B->user));
  const mcs_options& o = B->opt;
  const int prec = o.precision;
  std::vector<mcs_solve_info> inf(B->n);
  for (auto& v : inf) {
    v.status = MCS_OK;
    v.outer_steps = 1;
  }
  // load vectors b (union layout, FP64 slot VB64)
  for (auto& G : B->groups) {
    mcs_problem* u = G.u.get();
    const int64_t per = (int64_t)u->sz.nlat * u->d;
    for (int j = 0; j < G.np(); ++j)
      HIPCHK(hipMemcpyAsync(G.fun + u->pe0[j] * per, f[G.members[j]], (u->pe0[j + 1] - u->pe0[j]) * per * 8,
                            hipMemcpyDeviceToDevice, G.stream));
    int rc = mcs_load(u, G.fun, Ctx<double>(u).v(VB64));
    if (rc) return rc;
  }
  for (auto& G : B->groups) HIPCHK(hipStreamSynchronize(G.stream));
  auto t0 = std::chrono::steady_clock::now();
  // every member starts in the iteration
  for (auto& G : B->groups) {
    for (int j = 0; j < G.np(); ++j) G.h_int[2 * G.np() + j] = 1;
    HIPCHK(hipMemcpyAsync(G.act, G.h_int + 2 * G.np(), G.np() * 4, hipMemcpyHostToDevice, G.stream));
    HIPCHK(hipMemcpyAsync(G.go, G.h_int + 2 * G.np(), G.np() * 4, hipMemcpyHostToDevice, G.stream));
  }
  int rc = MCS_OK;
  if (prec == 0) {
    std::vector<GroupRun<double>> runs;
    for (auto& G : B->groups) {
      const int np = G.np();
      for (int j = 0; j < np; ++j) {
        G.h_st[ST_TOL * np + j] = o.tol;
        G.h_st[ST_ABS * np + j] = -1.0;
        G.h_st[ST_SB1 * np + j] = -1.0;
      }
      rc = upload_fields(G, {ST_TOL, ST_ABS, ST_SB1});
      if (rc) return rc;
      mcs_problem* u = G.u.get();
      runs.emplace_back(&G, o.max_it, Ctx<double>(u).v(VX));
    }
    for (auto& r : runs) r.start(r.c.v(VB64));
    for (auto& G : B->groups) {
      HIPCHK(hipEventRecord(G.ev_join, G.stream));
      HIPCHK(hipStreamWaitEvent(B->main, G.ev_join, 0));
    }
    rc = run_iterations<double>(B, runs, o.max_it);
    if (rc) return rc;
    for (auto& G : B->groups) {
      const int np = G.np();
      HIPCHK(hipMemcpyAsync(G.h_st, G.st, (size_t)ST_NFIELD * np * 8, hipMemcpyDeviceToHost, B->main));
      HIPCHK(hipMemcpyAsync(G.h_int, G.its, (size_t)np * 4, hipMemcpyDeviceToHost, B->main));
      HIPCHK(hipMemcpyAsync(G.h_int + np, G.status, (size_t)np * 4, hipMemcpyDeviceToHost, B->main));
    }
    HIPCHK(hipStreamSynchronize(B->main));
    for (auto& G : B->groups) {
      const int np = G.np();
      for (int j = 0; j < np; ++j) {
        mcs_solve_info& v = inf[G.members[j]];
        v.iterations = G.h_int[j];
        v.status = G.h_int[np + j];
        v.rel_precond_residual = G.h_st[ST_REL * np + j];
      }
    }
  } else {
    // FP32 inner MINRES inside FP64 refinement, per member
    struct MState {
      double beta0 = -1.0, rel = 1.0, rn = 0.0;
      int total = 0, outer = 0, status = MCS_OK;
      bool going = true;
    };
    std::vector<MState> ms(B->n);
    std::vector<GroupRun<float>> runs;
    for (auto& G : B->groups) {
      mcs_problem* u = G.u.get();
      Ctx<double> c64(u);
      const int64_t n = u->ndof;
      launch_fill<double>(G.stream, n, 0.0, c64.v(VX64));
      launch_axpby<double>(G.stream, n, 1.0, c64.v(VB64), 0.0, c64.v(VR64));
      Ctx<float> c32(u);
      runs.emplace_back(&G, o.max_it, c32.v(VX64));
    }
    int outer = 0;
    for (outer = 0; outer < o.max_outer; ++outer) {
      // ||r||^2 per going member
      for (auto& G : B->groups) {
        mcs_problem* u = G.u.get();
        Ctx<double> c64(u);
        SegDev S = G.seg(G.go, o.max_it);
        launch_seg_dot<double>(G.stream, S, c64.v(VR64), c64.v(VR64), ST_RN);
        HIPCHK(hipMemcpyAsync(G.h_st + (size_t)ST_RN * G.np(), G.st + (size_t)ST_RN * G.np(), G.np() * 8,
                              hipMemcpyDeviceToHost, G.stream));
      }
      for (auto& G : B->groups) HIPCHK(hipStreamSynchronize(G.stream));
      bool any = false;
      for (auto& G : B->groups) {
        const int np = G.np();
        for (int j = 0; j < np; ++j) {
          MState& m = ms[G.members[j]];
          int32_t& gflag = G.h_int[2 * np + j];
          gflag = m.going ? 1 : 0;
          if (!m.going) continue;
          const double rn = std::sqrt(G.h_st[ST_RN * np + j]);
          if (!std::isfinite(rn)) {
            m.status = MCS_ERR_NONFINITE;
            m.going = false;
            gflag = 0;
            continue;
          }
          if (rn == 0.0) {
            m.rel = 0.0;
            m.going = false;
            gflag = 0;
            continue;
          }
          m.rn = rn;
          G.h_st[ST_RN * np + j] = rn;
          G.h_st[ST_TOL * np + j] = o.inner_tol;
          G.h_st[ST_SB1 * np + j] = m.beta0 > 0 ? o.tol * m.beta0 / rn : -1.0;
          G.h_st[ST_ABS * np + j] = m.beta0 > 0 ? 0.25 * o.tol * m.beta0 / rn : -1.0;
          any = true;
        }
        rc = upload_fields(G, {ST_RN, ST_TOL, ST_SB1, ST_ABS});
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(G.go, G.h_int + 2 * np, np * 4, hipMemcpyHostToDevice, G.stream));
        HIPCHK(hipMemcpyAsync(G.act, G.h_int + 2 * np, np * 4, hipMemcpyHostToDevice, G.stream));
      }
      if (!any) break;
      for (size_t g = 0; g < B->groups.size(); ++g) {
        Group& G = B->groups[g];
        mcs_problem* u = G.u.get();
        Ctx<double> c64(u);
        Ctx<float> c32(u);
        SegDev S = G.seg(G.go, o.max_it);
        float* r32 = c32.v(VB64);
        launch_seg_scale_convert<double, float>(G.stream, S, c64.v(VR64), r32, ST_RN, 1, 0);
        runs[g].start(r32);
        HIPCHK(hipEventRecord(G.ev_join, G.stream));
        HIPCHK(hipStreamWaitEvent(B->main, G.ev_join, 0));
      }
      rc = run_iterations<float>(B, runs, o.max_it);
      if (rc) return rc;
      for (auto& G : B->groups) {
        const int np = G.np();
        HIPCHK(hipMemcpyAsync(G.h_st + (size_t)ST_BETA1 * np, G.st + (size_t)ST_BETA1 * np, np * 8,
                              hipMemcpyDeviceToHost, B->main));
        HIPCHK(hipMemcpyAsync(G.h_int, G.its, (size_t)np * 4, hipMemcpyDeviceToHost, B->main));
        HIPCHK(hipMemcpyAsync(G.h_int + np, G.status, (size_t)np * 4, hipMemcpyDeviceToHost, B->main));
      }
      HIPCHK(hipStreamSynchronize(B->main));
      for (auto& G : B->groups) {
        const int np = G.np();
        for (int j = 0; j < np; ++j) {
          MState& m = ms[G.members[j]];
          int32_t& gflag = G.h_int[2 * np + j];
          gflag = 0;
          if (!m.going) continue;
          const double b1 = G.h_st[ST_BETA1 * np + j];
          const int its = G.h_int[j], ist = G.h_int[np + j];
          if (m.beta0 < 0) m.beta0 = b1 * m.rn;
          m.rel = m.beta0 > 0 ? b1 * m.rn / m.beta0 : 0.0;
          m.total += its;
          m.outer = outer + 1;
          if (ist == MCS_ERR_NONFINITE || ist == MCS_ERR_BREAKDOWN) {
            m.status = ist;
            m.going = false;
            continue;
          }
          if (m.rel <= o.tol) {   // the current outer residual is small enough
            m.going = false;
            continue;
          }
          gflag = 1;
        }
        HIPCHK(hipMemcpyAsync(G.go, G.h_int + 2 * np, np * 4, hipMemcpyHostToDevice, G.stream));
        // x += rn d;  r = b - K x   (FP64, going members)
        mcs_problem* u = G.u.get();
        Ctx<double> c64(u);
        Ctx<float> c32(u);
        c64.set_mask(G.elem_prob, G.facet_prob, G.go);
        SegDev S = G.seg(G.go, o.max_it);
        launch_seg_scale_convert<float, double>(G.stream, S, c32.v(VX64), c64.v(VX64), ST_RN, 0, 1);
        c64.apply(c64.v(VX64), c64.v(VT64), 1 | 2 | 4);
        launch_seg_sub(G.stream, S, c64.v(VB64), c64.v(VT64), c64.v(VR64));
      }
    }
    for (auto& G : B->groups)
      for (int j = 0; j < G.np(); ++j) {
        MState& m = ms[G.members[j]];
        mcs_solve_info& v = inf[G.members[j]];
        v.iterations = m.total;
        v.outer_steps = std::max(1, m.outer);
        v.rel_precond_residual = m.rel;
        v.status = m.status;
        if (v.status == MCS_OK && m.rel > o.tol) v.status = MCS_ERR_NOT_CONVERGED;
      }
  }
  for (auto& G : B->groups) HIPCHK(hipStreamSynchronize(G.stream));
  HIPCHK(hipStreamSynchronize(B->main));
  auto t1 = std::chrono::steady_clock::now();
  const double tms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  // true residuals, pressure normalisation, copy-out
  for (auto& G : B->groups) {
    mcs_problem* u = G.u.get();
    const int np = G.np();
    Ctx<double> c64(u);
    double* x = prec == 0 ? c64.v(VX) : c64.v(VX64);
    double* b = c64.v(VB64);
    double* kx = c64.v(VT64);
    double* rr = c64.v(VR64);
    for (int j = 0; j < np; ++j) G.h_int[2 * np + j] = 1;
    HIPCHK(hipMemcpyAsync(G.act, G.h_int + 2 * np, np * 4, hipMemcpyHostToDevice, G.stream));
    c64.set_mask(G.elem_prob, G.facet_prob, G.act);
    SegDev S = G.seg(G.act, o.max_it);
    c64.apply(x, kx, 1 | 2 | 4);
    launch_seg_sub(G.stream, S, b, kx, rr);
    launch_seg_dot<double>(G.stream, S, rr, rr, ST_ALPHA);
    launch_seg_dot<double>(G.stream, S, b, b, ST_BB);
    HIPCHK(hipMemcpyAsync(G.h_st, G.st, (size_t)ST_NFIELD * np * 8, hipMemcpyDeviceToHost, G.stream));
    SolveParams P = solve_params(u);
    launch_batch_pmean(G.stream, P, np, G.pe0, u->p.rpmom, u->p.rpconst, x);
    const Sizes& s = u->sz;
    for (int j = 0; j < np; ++j) {
      const mcs_problem* q = B->singles[G.members[j]].get();
      double* dst = xo[G.members[j]];
      const int64_t ne = q->ne, nff = q->nff;
      HIPCHK(hipMemcpyAsync(dst, x + u->pe0[j] * s.nb, ne * s.nb * 8, hipMemcpyDeviceToDevice, G.stream));
      HIPCHK(hipMemcpyAsync(dst + q->off_f, x + u->off_f + u->pf0[j] * s.nfb, nff * s.nfb * 8, hipMemcpyDeviceToDevice,
                            G.stream));
      HIPCHK(hipMemcpyAsync(dst + q->off_p, x + u->off_p + u->pe0[j] * s.np, ne * s.np * 8, hipMemcpyDeviceToDevice,
                            G.stream));
    }
  }
  for (auto& G : B->groups) {
    HIPCHK(hipStreamSynchronize(G.stream));
    const int np = G.np();
    for (int j = 0; j < np; ++j) {
      mcs_solve_info& v = inf[G.members[j]];
      const double rn = G.h_st[ST_ALPHA * np + j], bn = G.h_st[ST_BB * np + j];
      v.rel_residual = bn > 0 ? std::sqrt(rn / bn) : std::sqrt(rn);
      v.t_solve_ms = tms;
    }
  }
  HIPCHK(hipGetLastError());
  rc = MCS_OK;
  for (int i = 0; i < B->n; ++i)
    if (inf[i].status != MCS_OK && rc == MCS_OK) {
      rc = inf[i].status;
      set_error("member %d: %s after %d iterations (rel %.3e)", i, mcs_status_string(rc), inf[i].iterations,
                inf[i].rel_precond_residual);
    }
  if (infos) std::copy(inf.begin(), inf.end(), infos);
  return rc;
}

}  // namespace

extern "C" {

int mcs_batch_solve(mcs_batch* B, const double* const* f, double* const* xo, mcs_solve_info* infos) {
  if (async_busy(B)) return MCS_ERR_STATE;
  return batch_solve(B, f, xo, infos);
}

int mcs_batch_solve_async(mcs_batch* B, const double* const* f, double* const* xo) {
  if (async_busy(B)) return MCS_ERR_STATE;
  if (!B || !B->ws || !B->condensed) {
    set_error("batch solve needs bind and condense first");
    return B ? MCS_ERR_STATE : MCS_ERR_ARG;
  }
  if (!f || !xo) {
    set_error("null force or solution array");
    return MCS_ERR_ARG;
  }
  for (int i = 0; i < B->n; ++i)
    if (!f[i] || !xo[i]) {
      set_error("member %d: null force or solution pointer", i);
      return MCS_ERR_ARG;
    }
  // the inputs are read once the bind stream's work so far has finished
  if (B->user) HIPCHK(hipStreamSynchronize(B->user));
  B->async_f.assign(f, f + B->n);
  B->async_x.assign(xo, xo + B->n);
  B->async_inf.assign(B->n, mcs_solve_info{});
  B->async_rc = MCS_OK;
  B->async_err.clear();
  B->async_state.store(1, std::memory_order_release);
  try {
    B->async_thread = std::thread([B] {
      hipSetDevice(B->device);
      const int rc = batch_solve(B, B->async_f.data(), B->async_x.data(), B->async_inf.data());
      B->async_rc = rc;
      if (rc) B->async_err = mcs_last_error();
      B->async_state.store(2, std::memory_order_release);
    });
  } catch (...) {
    B->async_state.store(0, std::memory_order_release);
    set_error("could not start the solve thread");
    return MCS_ERR_STATE;
  }
  return MCS_OK;
}

int mcs_batch_poll(const mcs_batch* B, int32_t* done) {
  if (!B || !done) {
    set_error("batch poll: null argument");
    return MCS_ERR_ARG;
  }
  const int st = B->async_state.load(std::memory_order_acquire);
  if (st == 0) {
    set_error("batch poll: no asynchronous solve was started");
    return MCS_ERR_STATE;
  }
  *done = st == 2 ? 1 : 0;
  return MCS_OK;
}

int mcs_batch_wait(mcs_batch* B, mcs_solve_info* infos) {
  if (!B) {
    set_error("batch wait: null batch");
    return MCS_ERR_ARG;
  }
  if (B->async_state.load(std::memory_order_acquire) == 0) {
    set_error("batch wait: no asynchronous solve was started");
    return MCS_ERR_STATE;
  }
  if (B->async_thread.joinable()) B->async_thread.join();
  if (infos) std::copy(B->async_inf.begin(), B->async_inf.end(), infos);
  const int rc = B->async_rc;
  if (rc) set_error("%s", B->async_err.c_str());
  B->async_state.store(0, std::memory_order_release);
  return rc;
}

int mcs_batch_launch_config(const mcs_batch* B, int32_t g, int dt, int32_t* dim, int32_t* order,
                            int32_t* facets_per_block, int64_t* grid_cap, double* us) {
  if (!B || g < 0 || g >= (int32_t)B->groups.size()) {
    set_error("batch launch config: bad group");
    return MCS_ERR_ARG;
  }
  const mcs_problem* u = B->groups[g].u.get();
  if (dim) *dim = u->d;
  if (order) *order = u->sz.k;
  return mcs_get_launch_config(u, dt, facets_per_block, grid_cap, us);
}

int mcs_batch_timer_enable(mcs_batch* B, int enable) {
  if (async_busy(B)) return MCS_ERR_STATE;
  if (!B || !B->ws) {
    set_error("batch is not bound");
    return B ? MCS_ERR_STATE : MCS_ERR_ARG;
  }
  for (auto& G : B->groups) {
    int rc = mcs_timer_enable(G.u.get(), enable);
    if (rc) return rc;
  }
  B->timer = enable != 0;
  return MCS_OK;
}

int mcs_batch_timer_read(mcs_batch* B, double* total_ms, int64_t* launches, double* bytes) {
  if (async_busy(B)) return MCS_ERR_STATE;
  if (!B || !B->ws) {
    set_error("batch is not bound");
    return B ? MCS_ERR_STATE : MCS_ERR_ARG;
  }
  double ms = 0.0, by = 0.0;
  int64_t n = 0;
  for (auto& G : B->groups) {
    double m = 0.0, b = 0.0;
    int64_t l = 0;
    int rc = mcs_timer_read(G.u.get(), MCS_TIMER_SMOOTH, &m, &l, &b);
    if (rc) return rc;
    ms += m;
    by += b;
    n += l;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (bytes) *bytes = by;
  return MCS_OK;
}

void mcs_batch_destroy(mcs_batch* B) {
  // an asynchronous solve still running is waited for (outside the API lock,
  // which the solve thread takes)
  if (B && B->async_thread.joinable()) B->async_thread.join();
  ApiLock lock(device_api_mutex());
  delete B;
}

}  // extern "C"
