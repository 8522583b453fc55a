// Solver context shared by the single-problem and batched drivers: work
// vector slots, kernel parameter blocks of a bound problem (or union of
// problems) and the host orchestration of the operators and preconditioner:
//   K-hat^{-1} (eq. mhatinvfactor) with two A-hat_ext^{-1} applications
//   (Sec. 6.1), A-hat^d_m^{-1} (Corollary aux_pc_mult: forward coloured block
//   Gauss-Seidel sweeps, coarse correction E^d C^{-1} E^d^T, backward sweeps),
//   C = one V(1,1) cycle on the P1 lattice hierarchy.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels_common.h"
#include "launch.h"

namespace mcs {

int64_t offset_of(const mcs_problem* pb, const char* name);

// work-vector slots
enum { VX = 0, VR1, VR2, VY, VV, VW1, VW2, VKV, PA1, PG, PS, PT, PT1, PTMP, PB1, VB64, VR64, VX64, VT64, PZ, NVEC };

template <typename T>
T* ws_ptr(mcs_problem* pb, const char* name) {
  int64_t off = offset_of(pb, name);
  return off < 0 ? nullptr : reinterpret_cast<T*>(static_cast<char*>(pb->ws) + off);
}

inline SolveParams solve_params(mcs_problem* pb) {
  SolveParams P{};
  P.s = pb->sz;
  P.ne = pb->ne;
  P.nff = pb->nff;
  P.off_f = pb->off_f;
  P.has_outlet = pb->has_outlet ? 1 : 0;
  P.off_p = pb->off_p;
  P.ndof = pb->ndof;
  P.elem_ff = pb->p.elem_ff;
  P.facet_el = pb->p.facet_el;
  P.facet_slot = pb->p.facet_slot;
  P.colour_desc = pb->p.colour_desc;
  P.detJ = pb->p.detJ;
  P.nu = pb->p.nu;
  P.rBp = pb->p.rBp;
  P.rMpinv = pb->p.rMpinv;
  return P;
}

template <typename R>
OpPtrs<R> op_ptrs(mcs_problem* pb);
template <>
inline OpPtrs<double> op_ptrs<double>(mcs_problem* pb) {
  return {pb->p.Ad, pb->p.H, pb->p.Aoo, pb->p.Aooinv, pb->p.Dinv, pb->p.EF, pb->p.W,
          pb->p.Ad32, pb->p.Adl, pb->p.H32, pb->p.Hl, pb->p.Aoo32, pb->p.Aool, pb->p.DinvP};
}
template <>
inline OpPtrs<float> op_ptrs<float>(mcs_problem* pb) {
  return {pb->p.Ad32, pb->p.H32, pb->p.Aoo32, pb->p.Aooinv32, pb->p.Dinv32, pb->p.EF32, pb->p.W32,
          nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, pb->p.DinvP32};
}

template <typename R>
std::vector<MGLevelDev> mg_levels(mcs_problem* pb) {
  std::vector<MGLevelDev> out;
  const int d = pb->d, st = d == 3 ? 27 : 9;
  char* base = static_cast<char*>(pb->ws);
  for (auto& M : pb->mg) {
    MGLevelDev L{};
    L.nblk = (int)M.blocks.size();
    L.ncont = M.ncont;
    L.blk = reinterpret_cast<const MGBlockDev*>(base + M.off_blk);
    L.maxv = M.maxv;
    L.maxvc = M.maxvc;
    L.maxnc = M.maxnc;
    size_t nA = (size_t)M.nvert * st * d * d, nD = (size_t)M.nvert * d * d;
    if (sizeof(R) == 8) {
      L.A = base + M.off_A;
      L.Dinv = base + M.off_Dinv;
    } else {
      L.A = base + M.off_A + nA * 8;
      L.Dinv = base + M.off_Dinv + nD * 8;
    }
    L.x = base + M.off_x;
    L.b = base + M.off_b;
    L.r = base + M.off_r;
    out.push_back(L);
  }
  return out;
}

// Algorithmic HBM bytes of one facet block of the smoother kernel with
// words of wsize bytes: the facet's rows of A^d_T of both neighbours
// (2 n_fb n_d), the packed upper triangle of D_F^{-1} (n_fb (n_fb + 1) / 2),
// the right-hand side and the updated block (3 n_fb), the neighbours'
// maintained products read and written (4 n_d), two more block reads
// (2 n_fb) and the 16-byte facet record.
inline double smooth_bytes_per_facet(const Sizes& z, int wsize) {
  return double(2 * z.nfb * z.nd + z.nfb * (z.nfb + 1) / 2 + 4 * z.nd + 5 * z.nfb) * wsize + 16.0;
}
// device counters of processed facet blocks: 256 counters (stride 16) for
// FP64 launches, then 256 for FP32 launches
constexpr int WCOUNT = 2 * 256 * 16;
inline unsigned long long* work_counters(mcs_problem* pb) { return pb->p.wcount; }

// Algorithmic bytes of one element of the operator apply K x (k_elem_apply
// with A, B^T p and B u): A^d_T, H_T and A_oo,T as stored (n_d^2 + n_b n_d +
// n_b^2 words), the gathered inputs and written outputs (2 (n_d + n_b + n_p)
// words), the free facet ids and det J.
inline double kapply_bytes_per_elem(const Sizes& z, int d, int wsize) {
  return double(z.nd * z.nd + z.nb * z.nd + z.nb * z.nb + 2 * (z.nd + z.nb + z.np)) * wsize + 4.0 * (d + 1) + 8.0;
}

// Accumulates the elapsed time of recorded (start, stop) event pairs; the
// caller has synchronised the stream.
inline void timer_flush(mcs_problem* pb) {
  for (size_t i = 0; i < pb->tpending; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pb->tev[2 * i], pb->tev[2 * i + 1]) == hipSuccess) pb->t_ms[pb->tkind[i]] += ms;
  }
  pb->tpending = 0;
}

// Records the start event of a timed launch of kernel `kind` on stream st.
inline void timer_start(mcs_problem* pb, hipStream_t st, int kind) {
  const size_t k = pb->tpending;
  while (pb->tev.size() < 2 * k + 2) {
    ApiLock lock(device_api_mutex());
    hipEvent_t e;
    hipEventCreate(&e);
    pb->tev.push_back(e);
  }
  if (pb->tkind.size() < k + 1) pb->tkind.resize(k + 1);
  pb->tkind[k] = kind;
  hipEventRecord(pb->tev[2 * k], st);
}

inline void timer_stop(mcs_problem* pb, hipStream_t st) {
  const int kind = pb->tkind[pb->tpending];
  hipEventRecord(pb->tev[2 * pb->tpending + 1], st);
  pb->tpending++;
  pb->t_launches[kind]++;
}

template <typename R>
struct Ctx {
  mcs_problem* pb;
  hipStream_t st;
  SolveParams P;
  OpPtrs<R> O;
  std::vector<MGLevelDev> L;
  R* base;
  R* escr;
  R* fscr;
  int64_t n;
  // device alias of the caller's pinned scalar (set by the solve driver): the
  // final reduction of a dot product writes there directly, so that reading a
  // scalar needs no copy launch
  double* host_dev = nullptr;
  // reduction partials (>= 1024 doubles) and the scalar slot of dot products
  double* red;
  double* scal;
  explicit Ctx(mcs_problem* p) : pb(p), st(p->stream), P(solve_params(p)), O(op_ptrs<R>(p)), L(mg_levels<R>(p)) {
    n = p->ndof;
    red = p->p.red;
    scal = p->p.scal;
    base = sizeof(R) == 8 ? reinterpret_cast<R*>(p->p.vec) - (int64_t)p->vbase64 * p->ndof
                          : reinterpret_cast<R*>(p->p.vec32);
    escr = reinterpret_cast<R*>(p->p.escr);
    fscr = reinterpret_cast<R*>(p->p.fscr);
    P.apply_rpt = p->tune_rpt[sizeof(R) == 8 ? 0 : 1];
  }
  R* v(int i) { return base + (int64_t)i * n; }

  // Restricts the work of every operator to the active members of a union.
  void set_mask(const int32_t* elem_prob, const int32_t* facet_prob, const int32_t* active) {
    P.elem_prob = elem_prob;
    P.facet_prob = facet_prob;
    P.active = active;
    for (auto& l : L) l.active = active;
  }

  // Element parts of the operator (escr, pressure rows of y) and of the
  // pressure block; the lowest order (no bubbles, one pressure dof) takes the
  // one-wave-per-element kernels.
  bool wave_elements() const { return pb->sz.nb == 0 && pb->sz.np == 1; }
  void elem_apply(const R* x, R* y, int flags) {
    if (wave_elements()) launch_elem_apply_wave<R>(st, P, O, x, y, escr, flags);
    else launch_elem_apply<R>(st, P, O, x, y, escr, flags);
  }
  void elem_press(const R* a, const R* r, R* y, int with_B) {
    if (wave_elements()) launch_elem_press_wave<R>(st, P, a, r, y, with_B);
    else launch_elem_press<R>(st, P, a, r, y, with_B);
  }

  // y = op x on full vectors; flags of k_elem_apply.
  void apply(const R* x, R* y, int flags) {
    if (flags & 8) launch_fill<R>(st, n, R(0), y);
    // the timer takes the full operator apply of a single problem (no masks),
    // in the precision of the MINRES iteration (precision 1: the FP32 applies,
    // not the FP64 ones of the refinement residual)
    const bool timed = pb->timer_on && flags == (1 | 2 | 4) && !P.active && (!pb->lean || sizeof(R) == 4) &&
                       pb->t_tick[1]++ % pb->timer_period == 0;
    if (timed) {
      timer_start(pb, st, 1);
      pb->t_bytes[1] += pb->ne * kapply_bytes_per_elem(pb->sz, pb->d, sizeof(R));
    }
    elem_apply(x, y, flags);
    if (timed) timer_stop(pb, st);
    launch_facet_sum<R>(st, P, escr, nullptr, R(1), y);
  }

  // One V(1,1) cycle from level l: blocks on their problem's coarsest level
  // are solved densely, the continuing ones smoothed and restricted.
  void vcycle(size_t l) {
    const int d = pb->d;
    if (L[l].ncont < L[l].nblk) launch_mg_coarse<R>(st, pb->p.Cinv, pb->p.cmap, d, L[l]);
    if (L[l].ncont == 0) return;
    launch_mg_point<R>(st, d, L[l], 0);
    launch_mg_point<R>(st, d, L[l], 1);
    launch_mg_restrict<R>(st, d, L[l], L[l + 1]);
    vcycle(l + 1);
    launch_mg_prolong<R>(st, d, L[l], L[l + 1]);
    // post-smoothing x += D^{-1} (b - A x): the residual first (mode 1 reads x,
    // writes r), then the pointwise update (mode 2), so that no launch reads
    // the x it writes
    launch_mg_point<R>(st, d, L[l], 1);
    launch_mg_point<R>(st, d, L[l], 2);
  }

  // `smoothing_steps` block Gauss-Seidel sweeps on A^d (colours ascending or
  // descending); y holds the element products A^d_T x_T and is kept current,
  // except by the very last colour phase when y_dead (the caller does not use
  // y afterwards): that phase only updates x (launch_smooth_last).
  void sweeps(R* x, const R* s, R* y, bool forward, bool y_dead = false) {
    SolveParams Pt = P;
    // the timer samples one call in timer_period (all launches of that call)
    const bool timed = pb->timer_on && pb->t_tick[0]++ % pb->timer_period == 0;
    if (timed) Pt.work_count = work_counters(pb) + (sizeof(R) == 8 ? 0 : 256 * 16);
    const int fpw = pb->tune_fpw[sizeof(R) == 8 ? 0 : 1];
    const int64_t cap = pb->tune_cap[sizeof(R) == 8 ? 0 : 1];
    for (int it = 0; it < pb->opt.smoothing_steps; ++it)
      for (int cc = 0; cc < pb->ncol; ++cc) {
        int c = forward ? cc : pb->ncol - 1 - cc;
        if (y_dead && it == pb->opt.smoothing_steps - 1 && cc == pb->ncol - 1) {
          launch_smooth_last<R>(st, P, O, pb->colour_off[c], pb->colour_off[c + 1], x, s, y);
          continue;
        }
        if (timed) {
          timer_start(pb, st, 0);
          launch_smooth_phase<R>(st, Pt, O, pb->colour_off[c], pb->colour_off[c + 1], x, s, y, fpw, cap);
          timer_stop(pb, st);
        } else {
          launch_smooth_phase<R>(st, P, O, pb->colour_off[c], pb->colour_off[c + 1], x, s, y, fpw, cap);
        }
      }
  }

  // z_d = E^d C^{-1} E^d^T r_d  (added to z if add)
  void aux(const R* r, R* z, int add) {
    launch_edt<R>(st, P, O, r, fscr, pb->nfv, pb->p.vinc_off, pb->p.vinc, pb->p.free_to_lat, (R*)L[0].b, 0);
    vcycle(0);
    launch_ed<R>(st, P, O, pb->p.facet_vfree, pb->p.free_to_lat, (const R*)L[0].x, z, add, 0);
  }

  // x = A-hat^d_m^{-1} s (facet parts; x fully overwritten):
  //   forward sweeps from x = 0; r = s - A^d x (from the maintained products);
  //   x += E^d C^{-1} E^d^T r (products updated through W_T); backward sweeps.
  // x = A-hat^d^{-1} s of the chosen variant: multiplicative (block
  // Gauss-Seidel sweeps around the coarse correction) or additive
  // (D^{-1} s + E^d C^{-1} E^d^T s with the facet block Jacobi D).
  void ad_inv(const R* s, R* x) {
    if (pb->opt.smoother == 3) {
      ad_l1_inv(s, x);
      return;
    }
    if (pb->opt.smoother == 1) {
      launch_fill<R>(st, n, R(0), x);
      launch_block_jacobi<R>(st, P, O, s, x);
      aux(s, x, 1);
      return;
    }
    ad_mult_inv(s, x);
  }

  void ad_mult_inv(const R* s, R* x) {
    R* tmp = v(PTMP);
    launch_fill<R>(st, n, R(0), x);
    launch_fill<R>(st, pb->ne * pb->sz.nd, R(0), escr);
    sweeps(x, s, escr, true);
    launch_facet_sum<R>(st, P, escr, s, R(-1), tmp);
    aux(tmp, x, 1);
    launch_ycorr<R>(st, P, O.W, pb->p.elem_verts, pb->p.vfree_of_lat, (const R*)L[0].x, escr);
    sweeps(x, s, escr, false, true);   // the products are not needed after the last phase
  }

  // x = A-hat^d^{-1} s of the l1 variant (smoother 3): facet block l1-Jacobi
  // sweeps x += M^{-1} (s - A^d x) (the facet blocks hold M_F^{-1}) around
  // the coarse correction; the element scratch keeps the products A^d_T x_T
  // (recomputed after a sweep, updated through W_T after the coarse
  // correction).  The first sweep from x = 0 is x = M^{-1} s.
  void ad_l1_inv(const R* s, R* x) {
    R *tmp = v(PTMP), *z = v(PZ);
    const int64_t of = pb->off_f, nf = (int64_t)pb->nff * pb->sz.nfb;
    const int steps = pb->opt.smoothing_steps;
    auto products = [&]() { elem_apply(x, tmp, 1 | 8); };
    auto sweep = [&]() {
      launch_facet_sum<R>(st, P, escr, s, R(-1), tmp);
      launch_block_jacobi<R>(st, P, O, tmp, z);
      launch_axpby<R>(st, nf, 1.0, z + of, 1.0, x + of);
    };
    launch_fill<R>(st, n, R(0), x);
    launch_block_jacobi<R>(st, P, O, s, x);
    for (int it = 1; it < steps; ++it) {
      products();
      sweep();
    }
    products();
    launch_facet_sum<R>(st, P, escr, s, R(-1), tmp);
    aux(tmp, x, 1);
    launch_ycorr<R>(st, P, O.W, pb->p.elem_verts, pb->p.vfree_of_lat, (const R*)L[0].x, escr);
    for (int it = 0; it < steps; ++it) {
      if (it > 0) products();
      sweep();
    }
  }

  FullDev full_dev() const {
    FullDev F{};
    F.nblk = pb->nblk;
    F.nbk = pb->sz.nfb + 2 * pb->sz.nb;
    F.blk_el = pb->p.blk_el;
    F.blk_slot = pb->p.blk_slot;
    F.blk_g = pb->p.blk_g;
    F.colour_blocks = pb->p.colour_blocks;
    F.A = pb->p.Afull;
    F.Binv = pb->p.Binv;
    F.W = pb->p.Wfull;
    F.Eo = pb->p.Eo;
    F.Eo_ref = pb->p.Eoref;
    return F;
  }

  // y = A-hat^{-1} r of the full-system variant (velocity parts; pressure
  // part of y set to 0): x = 0; forward overlapping block Gauss-Seidel
  // sweeps; coarse correction with the full embedding on r - A x; backward
  // sweeps.  FP64 only (the planner refuses other precisions).
  void full_inv(const R* r, R* y) {
    if constexpr (sizeof(R) == 8) {
      const FullDev F = full_dev();
      double* yf = pb->p.yfull;
      double* tmp = v(PTMP);
      launch_fill<R>(st, n, R(0), y);
      launch_fill<double>(st, pb->ne * pb->sz.nA, 0.0, yf);
      full_sweeps(F, y, r, yf, true);
      launch_full_resid(st, P, r, yf, tmp);
      launch_edt<R>(st, P, O, tmp, fscr, pb->nfv, pb->p.vinc_off, pb->p.vinc, pb->p.free_to_lat, (R*)L[0].b, 0);
      launch_full_edt(st, P, F, tmp, pb->p.eto, pb->nvert, pb->p.vert_elem_off, pb->p.vert_elem, pb->p.elem_verts,
                      pb->p.vfree_of_lat, (double*)L[0].b);
      vcycle(0);
      launch_ed<R>(st, P, O, pb->p.facet_vfree, pb->p.free_to_lat, (const R*)L[0].x, y, 1, 0);
      launch_full_ed(st, P, F, pb->p.elem_verts, pb->p.vfree_of_lat, (const double*)L[0].x, y, yf);
      full_sweeps(F, y, r, yf, false);
      launch_fill<R>(st, pb->ndof - pb->off_p, R(0), y + pb->off_p);
    }
  }

  void full_sweeps(const FullDev& F, double* x, const double* s, double* yf, bool forward) {
    const bool timed = pb->timer_on && pb->t_tick[0]++ % pb->timer_period == 0;
    for (int it = 0; it < pb->opt.smoothing_steps; ++it)
      for (int cc = 0; cc < pb->ncol_full; ++cc) {
        const int c = forward ? cc : pb->ncol_full - 1 - cc;
        if (timed) {
          timer_start(pb, st, 0);
          pb->t_bytes[0] += pb->full_colour_bytes[c];
        }
        launch_full_smooth(st, P, F, pb->colour_off_full[c], pb->colour_off_full[c + 1], x, s, yf);
        if (timed) timer_stop(pb, st);
      }
  }

  // y = A-hat_ext^{-1} r (velocity parts; pressure part of y set to 0); the
  // full-system variant replaces it by its own A-hat^{-1}
  void ext_inv(const R* r, R* y) {
    if (pb->opt.smoother == 2) {
      full_inv(r, y);
      return;
    }
    R *S = v(PS), *T = v(PT), *T1 = v(PT1);
    if (pb->sz.nb == 0) {
      ad_inv(r, T);   // no velocity bubbles (k = 1): A-hat_ext = A-hat^d
    } else {
      launch_ext_pre<R>(st, P, O, r, T1, escr);
      launch_facet_sum<R>(st, P, escr, r, R(-1), S);
      ad_inv(S, T);
      launch_ext_post<R>(st, P, O, T, T1, y);
    }
    launch_axpby<R>(st, pb->nff * pb->sz.nfb, 1.0, T + pb->off_f, 0.0, y + pb->off_f);
    launch_fill<R>(st, pb->ndof - pb->off_p, R(0), y + pb->off_p);
  }

  // z = K-hat^{-1} r:  a = A^{-1} r_u;  z_p = M_p^{-1}(r_p - B a);  z_u = a - A^{-1} B^T z_p
  void khat(const R* r, R* z) {
    R *A1 = v(PA1), *G = v(PG), *B1 = v(PB1);
    ext_inv(r, A1);
    elem_press(A1, r, z, 1);
    elem_apply(z, G, 2 | 16);
    launch_facet_sum<R>(st, P, escr, nullptr, R(1), G);
    ext_inv(G, B1);
    launch_axpby<R>(st, pb->off_p, 1.0, A1, 0.0, z);
    launch_axpby<R>(st, pb->off_p, -1.0, B1, 1.0, z);
  }

  double dot(const R* a, const R* b, double* host) {
    if (host_dev) {
      launch_dot<R>(st, n, a, b, red, host_dev);
    } else {
      launch_dot<R>(st, n, a, b, red, scal);
      hipMemcpyAsync(host, scal, sizeof(double), hipMemcpyDeviceToHost, st);
    }
    hipStreamSynchronize(st);
    timer_flush(pb);
    return *host;
  }

  // Preconditioned MINRES from x = 0 for K x = b.  Returns status.
  // Stops when ||r||_{K-hat^{-1}} <= max(tol * beta1, abs_stop); returns
  // immediately (0 iterations) when beta1 <= stop_beta1.
  int minres(const R* b, R* x, double tol, int maxit, double stop_beta1, double abs_stop, int* its, double* rel,
             double* beta1_out, double* host) {
    R *r1 = v(VR1), *r2 = v(VR2), *y = v(VY), *vv = v(VV), *w1 = v(VW1), *w2 = v(VW2), *kv = v(VKV);
    launch_fill<R>(st, n, R(0), x);
    launch_fill<R>(st, n, R(0), r1);
    launch_fill<R>(st, n, R(0), w1);
    launch_fill<R>(st, n, R(0), w2);
    launch_axpby<R>(st, n, 1.0, b, 0.0, r2);
    khat(r2, y);
    double b2 = dot(r2, y, host);
    *its = 0;
    if (!std::isfinite(b2)) return MCS_ERR_NONFINITE;
    if (b2 < 0) return MCS_ERR_BREAKDOWN;
    double beta1 = std::sqrt(b2);
    *beta1_out = beta1;
    *rel = 0.0;
    if (beta1 == 0.0 || beta1 <= stop_beta1) return MCS_OK;
    double beta = beta1, oldb = 0.0, dbar = 0.0, eps = 0.0, phibar = beta1, cs = -1.0, sn = 0.0;
    for (int it = 1; it <= maxit; ++it) {
      launch_axpby<R>(st, n, 1.0 / beta, y, 0.0, vv);
      apply(vv, kv, 1 | 2 | 4);
      if (it > 1) launch_axpby<R>(st, n, -beta / oldb, r1, 1.0, kv);
      double alpha = dot(vv, kv, host);
      launch_axpby<R>(st, n, -alpha / beta, r2, 1.0, kv);
      std::swap(r1, r2);   // r1 <- r2
      std::swap(r2, kv);   // r2 <- new residual, kv <- old r1 buffer (free)
      khat(r2, y);
      oldb = beta;
      double bb = dot(r2, y, host);
      if (!std::isfinite(bb) || !std::isfinite(alpha)) return MCS_ERR_NONFINITE;
      if (bb < 0) return MCS_ERR_BREAKDOWN;
      beta = std::sqrt(bb);
      double oldeps = eps;
      double delta = cs * dbar + sn * alpha;
      double gbar = sn * dbar - cs * alpha;
      eps = sn * beta;
      dbar = -cs * beta;
      double gamma = std::hypot(gbar, beta);
      if (gamma == 0.0) gamma = 1e-300;
      cs = gbar / gamma;
      sn = beta / gamma;
      double phi = cs * phibar;
      phibar = sn * phibar;
      launch_minres_w<R>(st, n, vv, w1, w2, x, 1.0 / gamma, -oldeps / gamma, -delta / gamma, phi);
      std::swap(w1, w2);
      *its = it;
      *rel = phibar / beta1;
      if (phibar <= std::max(tol * beta1, abs_stop)) return MCS_OK;
    }
    return MCS_ERR_NOT_CONVERGED;
  }
};


}  // namespace mcs
