// Request-level serving of MCS Stokes solves with continuous batching.
//
// Requests (mesh, order, viscosities, force) are queued on submit.  A
// scheduler thread takes waiting requests in arrival order into a
// micro-batch while their memory fits the free part of a caller-provided
// device arena (the HBM budget), and hands the micro-batch to a worker
// thread that runs it with the batch solver (mcs_batch_*): plan, bind,
// condense, solve, copy-out.  Up to max_inflight micro-batches run at the
// same time on their own streams, so requests that arrive while others are
// on the device start as soon as a slot and memory are free, and their work
// overlaps with the running ones.  A member's result does not depend on the
// other members of its batch, so every request gets the same answer alone
// or in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "mcs_internal.h"

namespace mcs {
const char* last_error();
}
using namespace mcs;

namespace {

using clk = std::chrono::steady_clock;

double ms_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over the arena (offsets, 4 KiB granularity).
struct Arena {
  size_t bytes = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  size_t used = 0, peak = 0;
  void init(size_t b) {
    bytes = b;
    free_.clear();
    free_[0] = b;
    used = peak = 0;
  }
  bool alloc(size_t n, size_t* off) {
    n = round_up(std::max<size_t>(n, 1), 4096);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        size_t rest = it->second - n, o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round_up(std::max<size_t>(n, 1), 4096);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
};

struct Request {
  int64_t id = 0;
  int dim = 3, order = 2;
  int32_t lattice[3] = {1, 1, 1};
  std::vector<double> vertices, nu, f;
  std::vector<int32_t> elements;
  size_t est_bytes = 0;     // workspace + io of the request alone
  int64_t ndof = 0;
  clk::time_point t_submit, t_start, t_done;
  bool done = false;
  std::vector<double> x;
  mcs_request_info info{};
  mcs_mesh mesh() const {
    mcs_mesh m{};
    m.dim = dim;
    m.n_vertices = (int32_t)(vertices.size() / dim);
    m.vertices_host = vertices.data();
    m.n_elements = (int32_t)(elements.size() / (dim + 1));
    m.elements_host = elements.data();
    for (int a = 0; a < 3; ++a) m.lattice[a] = lattice[a];
    return m;
  }
};

// device bytes of a batch's inputs and outputs: nu, f, x per member
size_t io_bytes(const std::vector<Request*>& rs, const std::vector<mcs_info>& infos) {
  size_t b = 0;
  for (size_t i = 0; i < rs.size(); ++i) {
    const Request* r = rs[i];
    const size_t ne = r->elements.size() / (r->dim + 1);
    b += round_up(ne * 8, 256) + round_up(r->f.size() * 8, 256) + round_up(infos[i].n_dof * 8, 256);
  }
  return b;
}

}  // namespace

struct mcs_server {
  mcs_options opt{};
  char* arena_ptr = nullptr;
  int device = 0;
  int max_inflight = 2, max_batch = 64;
  std::mutex mu;
  std::condition_variable cv;
  Arena arena;
  std::deque<Request*> waiting;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1;
  int inflight = 0;
  int64_t batches = 0, solved = 0;
  bool stop = false;
  std::thread scheduler;             // workers are detached; destroy waits for inflight == 0
  void run_scheduler();
  void run_batch(std::vector<Request*> rs, size_t off, size_t bytes);
};

void mcs_server::run_batch(std::vector<Request*> rs, size_t off, size_t bytes) {
  hipSetDevice(device);
  const int n = (int)rs.size();
  auto finish = [&](int status, const char* msg) {
    std::lock_guard<std::mutex> lk(mu);
    auto t = clk::now();
    for (auto* r : rs) {
      r->t_done = t;
      if (status != MCS_OK) {
        r->info.status = status;
        snprintf(r->info.message, sizeof(r->info.message), "%s", msg ? msg : "");
      }
      r->info.latency_ms = ms_between(r->t_submit, t);
      r->done = true;
    }
    arena.release(off, bytes);
    inflight--;
    solved += n;
    cv.notify_all();
  };
  std::vector<mcs_mesh> meshes(n);
  std::vector<int32_t> orders(n);
  for (int i = 0; i < n; ++i) {
    meshes[i] = rs[i]->mesh();
    orders[i] = rs[i]->order;
  }
  mcs_batch* b = nullptr;
  mcs_batch_info bi{};
  int rc = mcs_batch_plan(meshes.data(), orders.data(), n, &opt, &b, &bi);
  if (rc) return finish(rc, last_error());
  // the batch (streams, events, graphs) is destroyed before the reservation
  // is released
  std::unique_ptr<mcs_batch, void (*)(mcs_batch*)> guard(b, mcs_batch_destroy);
  auto done = [&](int status, const char* msg) {
    guard.reset();
    finish(status, msg);
  };
  std::vector<mcs_info> infos(n);
  for (int i = 0; i < n; ++i) mcs_batch_member_info(b, i, &infos[i]);
  char* base = arena_ptr + off;
  size_t ws = round_up(bi.workspace_bytes, 4096);
  if (ws + io_bytes(rs, infos) > bytes) return done(MCS_ERR_WORKSPACE, "batch larger than its reservation");
  rc = mcs_batch_bind(b, base, ws, nullptr);
  if (rc) return done(rc, last_error());
  std::vector<const double*> nu(n), f(n);
  std::vector<double*> x(n);
  char* io = base + ws;
  for (int i = 0; i < n; ++i) {
    Request* r = rs[i];
    const size_t ne = r->elements.size() / (r->dim + 1);
    double* dnu = reinterpret_cast<double*>(io);
    io += round_up(ne * 8, 256);
    double* df = reinterpret_cast<double*>(io);
    io += round_up(r->f.size() * 8, 256);
    double* dx = reinterpret_cast<double*>(io);
    io += round_up(infos[i].n_dof * 8, 256);
    bool up_ok;
    {
      ApiLock lock(device_api_mutex());
      up_ok = hipMemcpy(dnu, r->nu.data(), ne * 8, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(df, r->f.data(), r->f.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!up_ok) return done(MCS_ERR_HIP, "input upload failed");
    nu[i] = dnu;
    f[i] = df;
    x[i] = dx;
  }
  rc = mcs_batch_condense(b, nu.data());
  if (rc) return done(rc, last_error());
  std::vector<mcs_solve_info> si(n);
  rc = mcs_batch_solve(b, f.data(), x.data(), si.data());
  if (rc != MCS_OK && rc != MCS_ERR_NOT_CONVERGED && rc != MCS_ERR_BREAKDOWN && rc != MCS_ERR_NONFINITE)
    return done(rc, last_error());
  for (int i = 0; i < n; ++i) {
    Request* r = rs[i];
    r->x.resize(infos[i].n_dof);
    bool down_ok;
    {
      ApiLock lock(device_api_mutex());
      down_ok = hipMemcpy(r->x.data(), x[i], infos[i].n_dof * 8, hipMemcpyDeviceToHost) == hipSuccess;
    }
    if (!down_ok) return done(MCS_ERR_HIP, "result download failed");
    r->info.status = si[i].status;
    r->info.iterations = si[i].iterations;
    r->info.outer_steps = si[i].outer_steps;
    r->info.rel_residual = si[i].rel_residual;
    r->info.rel_precond_residual = si[i].rel_precond_residual;
    r->info.solve_ms = si[i].t_solve_ms;
    r->info.batch_size = n;
  }
  done(MCS_OK, "");
}

void mcs_server::run_scheduler() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    cv.wait(lk, [&] { return (stop && waiting.empty()) || (!waiting.empty() && inflight < max_inflight); });
    if (waiting.empty()) break;   // stop requested and nothing left to schedule
    // requests in arrival order while their standalone footprints fit the
    // largest free block (the union of several members needs at most the
    // sum of their standalone workspaces)
    const size_t avail = arena.largest();
    std::vector<Request*> take;
    size_t sum = 0;
    for (Request* r : waiting) {
      if ((int)take.size() >= max_batch) break;
      if (sum + r->est_bytes > avail) break;
      take.push_back(r);
      sum += r->est_bytes;
    }
    if (take.empty()) {
      Request* head = waiting.front();
      if (inflight == 0 && head->est_bytes > arena.bytes) {
        // can never fit: fail it
        waiting.pop_front();
        head->info.status = MCS_ERR_WORKSPACE;
        head->t_done = clk::now();
        head->info.latency_ms = ms_between(head->t_submit, head->t_done);
        head->done = true;
        cv.notify_all();
        continue;
      }
      cv.wait(lk, [&] { return inflight == 0 || arena.largest() >= head->est_bytes; });
      continue;
    }
    size_t off = 0;
    if (!arena.alloc(sum, &off)) continue;   // cannot happen: sum <= largest free block
    for (size_t i = 0; i < take.size(); ++i) waiting.pop_front();
    auto now = clk::now();
    for (Request* r : take) {
      r->t_start = now;
      r->info.queue_ms = ms_between(r->t_submit, now);
    }
    inflight++;
    batches++;
    std::thread(&mcs_server::run_batch, this, take, off, sum).detach();
  }
}

extern "C" {

int mcs_server_create(const mcs_options* options, void* arena, size_t arena_bytes, int32_t max_inflight,
                      int32_t max_batch, mcs_server** out) {
  if (!options || !arena || !out || arena_bytes < 4096 || (reinterpret_cast<uintptr_t>(arena) & 4095) ||
      max_inflight < 1 || max_batch < 1) {
    set_error("server: bad argument (arena must be 4096-byte aligned, limits >= 1)");
    return MCS_ERR_ARG;
  }
  std::unique_ptr<mcs_server> s(new (std::nothrow) mcs_server());
  if (!s) {
    set_error("out of host memory");
    return MCS_ERR_ARG;
  }
  s->opt = *options;
  s->arena_ptr = static_cast<char*>(arena);
  s->arena.init(arena_bytes);
  s->max_inflight = max_inflight;
  s->max_batch = max_batch;
  if (hipGetDevice(&s->device) != hipSuccess) {
    set_error("server: no HIP device");
    return MCS_ERR_HIP;
  }
  s->scheduler = std::thread(&mcs_server::run_scheduler, s.get());
  *out = s.release();
  return MCS_OK;
}

int mcs_server_submit(mcs_server* s, const mcs_mesh* mesh, int32_t order, const double* nu_host,
                      const double* f_host, int64_t* id) {
  if (!s || !mesh || !nu_host || !f_host || !id) {
    set_error("server submit: null argument");
    return MCS_ERR_ARG;
  }
  std::unique_ptr<Request> r(new Request());
  r->t_submit = clk::now();   // latency includes the planning below
  const int d = mesh->dim;
  r->dim = d;
  r->order = order;
  for (int a = 0; a < 3; ++a) r->lattice[a] = mesh->lattice[a];
  if ((d != 2 && d != 3) || mesh->n_vertices <= 0 || mesh->n_elements <= 0) {
    set_error("server submit: bad mesh");
    return MCS_ERR_ARG;
  }
  r->vertices.assign(mesh->vertices_host, mesh->vertices_host + (size_t)mesh->n_vertices * d);
  r->elements.assign(mesh->elements_host, mesh->elements_host + (size_t)mesh->n_elements * (d + 1));
  // footprint of the request alone (plan only: host work, no device memory)
  mcs_mesh m = r->mesh();
  mcs_batch* b = nullptr;
  mcs_batch_info bi{};
  int rc = mcs_batch_plan(&m, &order, 1, &s->opt, &b, &bi);
  if (rc) return rc;
  mcs_info mi{};
  mcs_batch_member_info(b, 0, &mi);
  mcs_batch_destroy(b);
  const int nlat = mi.n_lat;
  r->nu.assign(nu_host, nu_host + mesh->n_elements);
  r->f.assign(f_host, f_host + (size_t)mesh->n_elements * nlat * d);
  r->ndof = mi.n_dof;
  r->est_bytes = round_up(bi.workspace_bytes, 4096) +
                 round_up(mesh->n_elements * 8, 256) + round_up(r->f.size() * 8, 256) + round_up(mi.n_dof * 8, 256);
  r->info.status = 1;   // pending
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  *id = r->id;
  s->waiting.push_back(r.get());
  s->reqs[r->id] = std::move(r);
  s->cv.notify_all();
  return MCS_OK;
}

int mcs_server_poll(mcs_server* s, int64_t id, int32_t* done) {
  if (!s || !done) {
    set_error("server poll: null argument");
    return MCS_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    set_error("server poll: unknown request %lld", (long long)id);
    return MCS_ERR_ARG;
  }
  *done = it->second->done ? 1 : 0;
  return MCS_OK;
}

int mcs_server_wait(mcs_server* s, int64_t id, double* x_host, mcs_request_info* info) {
  if (!s) {
    set_error("server wait: null server");
    return MCS_ERR_ARG;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    set_error("server wait: unknown request %lld", (long long)id);
    return MCS_ERR_ARG;
  }
  Request* r = it->second.get();
  s->cv.wait(lk, [&] { return r->done; });
  if (x_host && !r->x.empty()) std::memcpy(x_host, r->x.data(), r->x.size() * 8);
  if (info) *info = r->info;
  const int st = r->info.status;
  s->reqs.erase(it);
  if (st != MCS_OK) set_error("request %lld: %s", (long long)id, mcs_status_string(st));
  return st;
}

int mcs_server_stats(mcs_server* s, mcs_server_stats_t* out) {
  if (!s || !out) {
    set_error("server stats: null argument");
    return MCS_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  out->arena_bytes = s->arena.bytes;
  out->arena_used = s->arena.used;
  out->arena_peak = s->arena.peak;
  out->batches = s->batches;
  out->solved = s->solved;
  out->waiting = (int64_t)s->waiting.size();
  out->inflight = s->inflight;
  return MCS_OK;
}

void mcs_server_destroy(mcs_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->scheduler.joinable()) s->scheduler.join();
  {
    // the scheduler has stopped launching; wait for the running batches
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->inflight == 0; });
  }
  delete s;
}

}  // extern "C"
