// Internal declarations of the MCS solver library (host + device).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcs.h"

namespace mcs {

void set_error(const char* fmt, ...);

// Host calls that may synchronise implicitly with other streams of the device
// (creating and releasing streams, events, graphs and pinned memory,
// synchronous copies) take this process-wide lock, and so does every stream
// capture, so that no capture in one thread overlaps such a call from
// another thread.  Recursive: batch binding binds its member problems.
std::recursive_mutex& device_api_mutex();
using ApiLock = std::lock_guard<std::recursive_mutex>;

// ---------------------------------------------------------------------------
// Local sizes of the spaces (Sec. 3) for dimension d and order k.
// ---------------------------------------------------------------------------
struct Sizes {
  int d, k, m;        // dimension, order, lattice degree of f
  int nv;             // d + 1 vertices
  int ns, nsm1;       // dim P^k(T), dim P^{k-1}(T)
  int nFk, nFkm1;     // dim P^k(F), dim P^{k-1}(F)
  int nu, nb, nF, nh, nfb, nd, nA, np;  // BDM, bubbles, facet normal, facet tangential, block, A^d, A, pressure
  int nw;             // omega flux dofs per facet: 1 for k = 1 (W_h in H(div), Sec. 7), else 0
  int nsym, nskew;    // orthonormal trace-free basis: symmetric / skew parts
  int sklo;           // first psi_a of the skew stress columns: nsm1 (omega in P^{k-1}(T, K)
                      // condensed), 0 for k = 1 (omega global)
  int nsig;           // reduced sigma columns: nsym * ns + nskew * (ns - sklo)
  int nlam;           // nt-degree constraints: (d+1)(d-1)(nFk - nFkm1)
  int nlat;           // lattice points of degree m
};
Sizes make_sizes(int d, int k);

// ---------------------------------------------------------------------------
// Reference-element tables (host computed once per (d, k), uploaded).
// All integrals are over the reference simplex T^ = conv{0, e_1..e_d} or its
// facets, with the reference measure.  Basis conventions:
//   phi^_i (BDM, n_u): bubbles first, lambda^alpha (e_a - e_s0); then facet f
//     functions (-1)^f (d-1)! lambda^beta (e_j0 - e_f).  Physical:
//     bubbles J phi^, facet functions J phi^ / det J.
//   psi^_a (n_s): L2(T^)/|T^|-orthonormal, degree graded (first nsm1 span P^{k-1}).
//   q^ (facet, nFk - nFkm1): L2(F^)/|F^|-orthonormal basis of P^k(F) minus P^{k-1}(F).
//   pressure lambda^gamma, |gamma| = k-1; lattice Lagrange L^_l (sorted order).
// ---------------------------------------------------------------------------
struct RefTables {
  Sizes s;
  std::vector<double> V;     // [nu][ns][d][d]      int psi_a d_s phi_{i,r}
  std::vector<double> Bf;    // [nv][nu][ns][d]     int_{F_f} psi_a phi_{i,r}
  std::vector<double> U;     // [nv][nFkm1][ns]     int_{F_f} psi_a lambda_F^gamma
  std::vector<double> L;     // [nv][nq][ns]        int_{F_f} q_q psi_a
  std::vector<double> D;     // [nu][nu]            int div phi_i div phi_j
  std::vector<double> Bp;    // [np][nu]            int div phi_i lambda^gamma_q
  std::vector<double> Mp;    // [np][np]            int lambda^gamma lambda^gamma'
  std::vector<double> Mpinv; // [np][np]
  std::vector<double> Rf;    // [nlat][nu][d]       int L_l phi_{i,r}
  std::vector<int32_t> latmap; // [(d+1)!][nlat]   caller lattice index -> sorted lattice index
  std::vector<double> cn;    // [nFk][d]            lambda_v (facet vertex v) in degree-k facet Bernstein
  std::vector<double> ct;    // [nFkm1][d]          lambda_v in degree k-1 facet Bernstein
                             //                     (k = 1: its facet mean 1/d, the projection Pi^0)
  std::vector<double> Lam;   // [ns][nv]            int_T^ psi_a lambda_j
  std::vector<double> pconst;// [np]                coefficients of p = 1
  std::vector<double> pmom;  // [np]                int_T^ lambda^gamma / |T^|
  std::vector<double> phi;   // [nu][nv + 3]        BDM function i: alpha (nv), reference vector w (3)
  std::vector<double> pidx;  // [np][nv]            pressure multi-indices gamma
  std::vector<double> Eo;    // [nv][d][nb]         bubble coefficients of lambda_v e_r
  std::vector<double> psi;   // [ns][ns]            psi_a = sum_j psi[a][j] lambda^{beta_j}
  std::vector<double> psib;  // [ns][nv]            degree-k multi-indices beta_j
  double facet_measure[4];   // |F^_f|
};
RefTables build_ref_tables(int d, int k);
int perm_index(const int* perm, int nv);   // rank of a permutation of 0..nv-1

// ---------------------------------------------------------------------------
// Multigrid.  Every problem has its own lattice hierarchy (fine .. coarsest);
// a union of problems keeps, per level, one lattice block per problem that
// still has that level.  Blocks whose problem continues to a coarser level
// are smoothed and restricted there; a block on its problem's coarsest level
// is solved densely.
// ---------------------------------------------------------------------------
struct LatLevel {
  int n[3];           // intervals per axis (n[2] = 0 in 2D)
  int64_t nvert;      // lattice vertices (incl. boundary)
  int64_t nfree;      // free dofs
};

struct MGBlock {
  int prob;
  int ffm = 0;                  // outlet faces of the problem (see lat_free)
  int n[3];
  int64_t nvert, voff;          // vertices, first vertex in the level arrays
  int coarsest;
  int nc3[3];                   // continuing: intervals of the next level
  int64_t nvert_c, cvoff;       // continuing: next-level vertices and offset
  int64_t nc, cmap_off, cinv_off;  // coarsest: free dofs, offsets in cmap / Cinv
};

struct MGLevel {
  int64_t nvert;                // all blocks of the level
  std::vector<MGBlock> blocks;  // continuing blocks first, then coarsest ones
  int ncont;
  int64_t maxv, maxvc, maxnc;   // largest block: vertices, next-level vertices, coarse dofs
  int64_t off_A, off_Dinv, off_x, off_b, off_r, off_blk;   // workspace offsets (bytes)
};

// Device pointers of one problem (all inside the caller workspace).
struct DevPtrs {
  // topology
  int32_t* elem_ff;       // [ne][nv] free facet id or -1
  int32_t* elem_verts;    // [ne][nv] sorted global vertex ids
  int32_t* elem_perm;     // [ne] permutation rank of sorted order w.r.t. caller order
  int32_t* facet_el;      // [nff][2] neighbour elements (ascending; -1: none, outlet facets)
  int32_t* facet_out;     // [nff] 1 for an outlet facet
  double* xD;             // [ne][nd] Dirichlet dofs of the element's Dirichlet facets
  int32_t* facet_slot;    // [nff][2] local facet index in each neighbour
  int32_t* colour_desc;   // [nff][4] facets sorted by colour: g, e1, e2, s1 | s2 << 8
  int32_t* facet_vfree;   // [nff][d] free P1 vertex ids of the facet's sorted vertices (-1)
  int32_t* vinc_off;      // [nfv+1] free vertex -> incident (facet, slot) CSR
  int32_t* vinc;          // [ninc][2]
  int32_t* vert_elem_off; // [nvert+1] lattice vertex -> incident elements CSR
  int32_t* vert_elem;     // [nve]
  double* coords;         // [nvert][d]
  int32_t* vfree_of_lat;  // [nvert] lattice vertex -> free P1 vertex or -1
  int32_t* free_to_lat;   // [nfv] free P1 vertex -> lattice vertex
  // reference tables
  double *rV, *rBf, *rU, *rL, *rD, *rLam, *rBp, *rMp, *rMpinv, *rRf, *rcn, *rct, *rpconst, *rpmom, *rphi, *rpidx, *rpsi, *rpsib;
  int32_t* rlatmap;
  // element operators
  double *nu, *detJ;
  double *Ad, *H, *Aoo, *Aooinv;
  float *Ad32, *H32, *Aoo32, *Aooinv32;
  double *Dinv, *EF, *W;
  float *Dinv32, *EF32, *W32;
  double* DinvP;            // D_F^{-1} upper triangles, row-major packed (colour phases)
  float* DinvP32;
  float *Adl, *Hl, *Aool;   // low parts of the split storage (lean layout)

  double* adtmp;            // per-slot FP64 A^d buffer of the condensation (lean layout)
  // multigrid coarsest
  double* Cinv;           // [nc][nc]
  int32_t* cmap;          // [nc] coarsest free dof -> lattice dof index
  // scratch
  double* cscratch;       // condensation scratch (slots)
  double* escr;           // [ne][nd] element vector scratch (double, reused as float)
  double* escr2;          // [ne][nd]
  double* fscr;           // [nff][d*d]
  double* red;            // reduction partials
  double* scal;           // scalar block (256 doubles)
  unsigned long long* wcount;  // smoother work counters (measurement)
  // full-system variant (smoother 2)
  int32_t *blk_el, *blk_slot, *blk_g, *colour_blocks;
  double *Afull, *Binv, *Wfull, *Eo, *Eoref;
  double* yfull;          // [ne][nA] maintained products A_T x_T
  double* eto;            // [ne][(d+1)d] bubble part of E^T r
  double* vec;            // MINRES / preconditioner work vectors (FP64), nvec64 * ndof
  float* vec32;           // FP32 work vectors, nvec32 * ndof
  double* p1;             // P1 work vectors (FP64) 4 * np1
  float* p132;            // P1 work vectors FP32
};

}  // namespace mcs

struct mcs_problem {
  mcs::Sizes sz;
  mcs_options opt;
  int d;
  int64_t ne, nvert, nff, nfv;          // elements, vertices, free facets, free vertices
  int lattice[3];
  int ncol;
  std::vector<int32_t> colour_off;      // [ncol+1]
  std::vector<int32_t> h_colour;        // [nff] colour of facet
  std::vector<int32_t> h_colour_facets, h_elem_ff, h_elem_verts, h_elem_perm, h_facet_el,
      h_facet_slot, h_facet_vfree, h_vinc_off, h_vinc, h_vert_elem_off, h_vert_elem,
      h_vfree_of_lat, h_free_to_lat;
  std::vector<double> h_coords;
  // full-system variant: one overlapping block per facet of the mesh in
  // canonical facet order, coloured so that facets of one element differ
  int64_t nblk = 0;
  int ncol_full = 0;
  // boundary conditions: outlet faces of each member problem (bits as in
  // lat_free), whether some facet is an outlet (then p is unique), and the
  // outlet flag of every free facet
  std::vector<int> pffm{0};
  bool has_outlet = false;
  bool has_dirichlet = false;   // mcs_set_dirichlet was called (xD holds g's dofs)
  std::vector<int32_t> h_facet_out;
  std::vector<int32_t> h_blk_el, h_blk_slot, h_blk_g, h_blk_colour, colour_off_full, h_colour_blocks;
  std::vector<double> full_colour_bytes;  // algorithmic bytes of one colour phase (FP64)
  mcs::RefTables ref;
  std::vector<mcs::MGLevel> mg;         // fine .. coarsest over all member problems
  int64_t nc;                            // coarsest free dofs, summed over problems
  int64_t ncinv;                         // sum of nc_i^2 (dense coarse inverses)
  std::vector<int32_t> h_cmap;           // per problem: coarsest free dof -> block-local lattice dof
  // member problems (one for a single problem; several for a union of
  // problems with the same dimension and order)
  int nprob = 1;
  std::vector<int64_t> pe0, pf0, pv0, pfv0;   // [nprob+1] element / free facet / vertex / free vertex offsets
  std::vector<std::vector<mcs::LatLevel>> plev;  // per problem: lattice hierarchy
  std::vector<std::vector<int32_t>> pcmap;      // per problem: coarsest free dof -> local lattice dof
  int64_t ndof, off_f, off_p, np1;
  int64_t n_slots;                       // condensation workgroup slots
  int64_t slot_doubles;
  int64_t nred;
  int nvec64, nvec32;
  // Lean layout (precision 1): A^d, H, A_oo stored once as FP32 hi + lo; no
  // FP64 preconditioner data; FP64 work vectors only for the refinement,
  // slots vbase64 .. vbase64 + nvec64 - 1.
  bool lean = false;
  int vbase64 = 0;
  size_t ws_bytes;
  // binding
  void* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = -1;
  bool condensed = false;
  mcs::DevPtrs p;
  // launch shape of the smoother colour phase per work precision [FP64, FP32]
  // (set by the autotuner; every shape gives the same result)
  int tune_fpw[2] = {1, 1};
  int64_t tune_cap[2] = {0, 0};
  double tune_us[2] = {0.0, 0.0};
  bool tune_fixed[2] = {false, false};   // set by the caller: autotuning leaves the slot alone
  // rows of A^d per thread of the operator apply per work precision (0: the
  // default choice), its tuned time per launch, and the caller's pin
  int tune_rpt[2] = {0, 0};
  double tune_rpt_us[2] = {0.0, 0.0};
  bool tune_rpt_fixed[2] = {false, false};
  // kernel timer: [0] smoother phase launches, [1] K apply launches
  bool timer_on = false;
  int timer_period = 1;               // time one call in timer_period
  int64_t t_tick[2] = {0, 0};         // calls seen per kernel kind
  std::vector<hipEvent_t> tev;        // pairs (start, stop)
  std::vector<int> tkind;             // timed kernel of each pending pair
  size_t tpending = 0;
  double t_ms[2] = {0.0, 0.0}, t_bytes[2] = {0.0, 0.0};
  int64_t t_launches[2] = {0, 0};
  ~mcs_problem() {
    for (auto e : tev) hipEventDestroy(e);
  }
  std::vector<std::pair<std::string, int64_t>> offsets;  // name -> byte offset
};

namespace mcs {
// Dirichlet dofs ([n_e][n_d], element-local facet order) of g given on the
// element lattices (caller vertex order); see mcs_set_dirichlet.
void dirichlet_lift(const mcs_problem* pb, const double* g_lattice, std::vector<double>& xD);
}  // namespace mcs
