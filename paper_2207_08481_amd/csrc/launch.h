// Host-side launch wrappers of the solve kernels (defined in kernels_solve.hip).
#pragma once
#include "kernels_common.h"

namespace mcs {

template <typename R>
void launch_elem_apply(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* x, R* y, R* escr, int flags);
int apply_h_lanes(int nd, int rows_per_thread);
bool apply_col_split(int nd, int rows_per_thread);
template <typename R>
void launch_facet_sum(hipStream_t st, const SolveParams& P, const R* escr, const R* base, R sign, R* y);
template <typename R>
void launch_ext_pre(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* r, R* to, R* escr);
template <typename R>
void launch_ext_post(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* t, const R* to, R* y);
template <typename R>
void launch_smooth_phase(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, int32_t c0, int32_t c1, R* x,
                         const R* s, R* y, int facets_per_block = 1, int64_t grid_cap = 0);
int smooth_team_threads(int nd);
// Assembled diagonal of A^d on the facet dofs (diag) and the l1 terms of the
// facet block l1-Jacobi smoother (l1), both [free facet][n_fb] doubles.
void launch_l1_terms(hipStream_t st, const FacetSetupParams& P, double* diag, double* l1);
// The last colour phase when the element products are not needed afterwards
// (x only; bitwise the x of launch_smooth_phase).
template <typename R>
void launch_smooth_last(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, int32_t c0, int32_t c1, R* x,
                        const R* s, const R* y);
template <typename R>
void launch_block_jacobi(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* r, R* z);
template <typename R>
void launch_ycorr(hipStream_t st, const SolveParams& P, const R* W, const int32_t* elem_verts,
                  const int32_t* vfree_of_lat, const R* x0, R* y);
template <typename R>
void launch_edt(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* r, R* fscr, int64_t nfv,
                const int32_t* vinc_off, const int32_t* vinc, const int32_t* free_to_lat, R* b, int compact);
template <typename R>
void launch_ed(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const int32_t* facet_vfree,
               const int32_t* free_to_lat, const R* x0, R* y, int add, int compact);
template <typename R>
void launch_mg_point(hipStream_t st, int d, const MGLevelDev& L, int mode);
template <typename R>
void launch_mg_restrict(hipStream_t st, int d, const MGLevelDev& F, const MGLevelDev& C);
template <typename R>
void launch_mg_prolong(hipStream_t st, int d, const MGLevelDev& F, const MGLevelDev& C);
template <typename R>
void launch_mg_coarse(hipStream_t st, const double* Cinv, const int32_t* cmap, int d, const MGLevelDev& L);
template <typename R>
void launch_elem_press(hipStream_t st, const SolveParams& P, const R* a, const R* r, R* y, int with_B);
// the same two operations for k = 1 (no bubbles, n_p = 1): one wave per element
template <typename R>
void launch_elem_apply_wave(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* x, R* y, R* escr,
                            int flags);
template <typename R>
void launch_elem_press_wave(hipStream_t st, const SolveParams& P, const R* a, const R* r, R* y, int with_B);
template <typename R>
void launch_axpby(hipStream_t st, int64_t n, double a, const R* x, double b, R* y);
template <typename R>
void launch_fill(hipStream_t st, int64_t n, R v, R* y);
template <typename A, typename B>
void launch_convert(hipStream_t st, int64_t n, const A* x, B* y);
template <typename R>
void launch_dot(hipStream_t st, int64_t n, const R* x, const R* y, double* part, double* out);

template <typename R>
void launch_minres_w(hipStream_t st, int64_t n, const R* v, R* w1, const R* w2, R* x, double a, double b, double c,
                     double phi);
template <typename A, typename B>
void launch_scale_convert(hipStream_t st, int64_t n, double a, const A* x, B* y, int add);

template <typename R>
void launch_scatter_compact(hipStream_t st, int64_t nfv, int d, const int32_t* f2l, const R* c, R* lat);
template <typename R>
void launch_gather_compact(hipStream_t st, int64_t nfv, int d, const int32_t* f2l, const R* lat, R* c);

// setup (kernels_setup.hip)
void launch_condense(hipStream_t st, const CondParams& P, int nslots);
void launch_stress(hipStream_t st, const StressParams& S, int nslots);
void launch_full_smooth(hipStream_t st, const SolveParams& P, const FullDev& F, int c0, int c1, double* x,
                        const double* sv, double* y);
void launch_full_resid(hipStream_t st, const SolveParams& P, const double* sv, const double* y, double* r);
void launch_full_edt(hipStream_t st, const SolveParams& P, const FullDev& F, const double* r, double* eto,
                     int64_t nvert, const int32_t* vert_elem_off, const int32_t* vert_elem, const int32_t* elem_verts,
                     const int32_t* vfree_of_lat, double* b);
// x_o += E_o x0 (bubble rows of the embedding) and y += W x0
void launch_full_ed(hipStream_t st, const SolveParams& P, const FullDev& F, const int32_t* elem_verts,
                    const int32_t* vfree_of_lat, const double* x0, double* x, double* y);
void launch_full_setup(hipStream_t st, const Sizes& s, int64_t ne, const FullDev& F, const int32_t* elem_verts,
                       const double* coords, const int32_t* elem_ff, const double* EF, int* status);
void launch_facet_setup(hipStream_t st, const FacetSetupParams& P);
void launch_wsetup(hipStream_t st, const FacetSetupParams& P, const int32_t* elem_ff, int64_t ne, double* W, float* W32);
void launch_p1_assemble(hipStream_t st, const P1Params& P);
void launch_mg_l1(hipStream_t st, const MGSetupParams& P);
void launch_mg_rap(hipStream_t st, const MGSetupParams& P);
void launch_coarse(hipStream_t st, const MGSetupParams& P, int jb, int nj, int64_t base, double* scratch,
                   double* Cinv, int* status);
void launch_to_f32(hipStream_t st, const double* a, float* b, int64_t n);
void launch_load(hipStream_t st, const CondParams& C, const SolveParams& P, const int32_t* elem_perm,
                 const int32_t* latmap, const double* rRf, const double* f, double* b, double* escr);
void launch_check_nu(hipStream_t st, const double* nu, int64_t n, int* status);
void launch_pressure_mean(hipStream_t st, const SolveParams& P, const double* pmom, const double* pconst, double* x,
                          double* red);

void launch_eval(hipStream_t st, const SolveParams& P, const double* coords, const int32_t* elem_verts,
                 const int32_t* elem_perm, const double* rphi, const double* rpidx, int npts, const double* pts,
                 const double* x, double* u, double* p);

// batched MINRES (kernels_batch.hip)
template <typename R>
void launch_seg_dot(hipStream_t st, const SegDev& S, const R* a, const R* b, int field);
template <typename R>
void launch_seg_scale(hipStream_t st, const SegDev& S, const R* src, R* dst, int field, int inv);
template <typename R>
void launch_seg_axpy_ratio(hipStream_t st, const SegDev& S, const R* x, R* y, int num, int den, int min_its);
template <typename R>
void launch_seg_w(hipStream_t st, const SegDev& S, const R* v, R* w1, const R* w2, R* x);
template <typename A, typename B>
void launch_seg_scale_convert(hipStream_t st, const SegDev& S, const A* x, B* y, int field, int inv, int add);
void launch_seg_sub(hipStream_t st, const SegDev& S, const double* a, const double* b, double* y);
void launch_mr_init(hipStream_t st, const SegDev& S);
void launch_mr_update(hipStream_t st, const SegDev& S);
void launch_mr_retire(hipStream_t st, const SegDev& S);
void launch_batch_pmean(hipStream_t st, const SolveParams& P, int nprob, const int64_t* pe0, const double* pmom,
                        const double* pconst, double* x);

}  // namespace mcs
