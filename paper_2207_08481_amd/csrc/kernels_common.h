// Kernel parameter blocks shared by the setup and solve kernels.
#pragma once
#include "mcs_internal.h"

namespace mcs {

constexpr int MAXND = 256;   // max A^d size (k = 5, 3D: 204)
constexpr int MAXNB = 96;    // max bubbles (84)
constexpr int MAXNP = 40;    // max pressure dofs (35)
// C of the tangential penalty nu C k^2 / h on outlet facets in A-bar (Lemma
// outflow asks for C large enough; with 8 the excess of E^d^T A^d E^d over
// A-bar stays below 1 % on the tested meshes, k = 2..4)
constexpr double OUTLET_PENALTY = 8.0;
constexpr int MAXNFB = 64;   // max facet block (51)

struct CondParams {
  Sizes s;
  int64_t ne;
  int64_t slot_doubles;
  const int32_t* elem_verts;
  const double* coords;
  const double* nu;
  const double *rV, *rBf, *rU, *rL, *rD;
  const double* rLam;   // [ns][nv] int_T^ psi_a lambda_j (k = 1: the omega rows of G)
  double facet_measure[4];
  double* scratch;
  double* detJ;
  double *Ad, *H, *Aoo, *Aooinv;
  float *Ad32, *H32, *Aoo32, *Aooinv32;
  // split storage (FP32 work precision with FP64 refinement): the FP64
  // arrays Ad, H, Aoo, Aooinv are absent; hi = the FP32 copy, lo = the FP32
  // rounding of the remainder, so hi + lo reproduces the FP64 value to ~2^-48.
  // A^d is formed in a per-slot FP64 buffer adtmp first.
  float *Adl, *Hl, *Aool;
  double* Afull;                 // optional: A_T itself (full-system variant)
  const int32_t* elem_ff;        // element -> free facet id (-1: Dirichlet)
  const int32_t* facet_out;      // free facet -> 1 for an outlet facet
  double* adtmp;
  int64_t adtmp_stride;
  int* status;
};

// Stress and vorticity recovery (eq. projection) at reference points.
struct StressParams {
  CondParams C;                  // geometry, reference tables, nu, slot scratch
  const double* x;               // global coefficient vector
  const int32_t* elem_ff;
  const int32_t* elem_perm;
  int64_t off_f;
  const double *rpsi, *rpsib;    // psi_a in monomial form, multi-indices
  const double* xD;              // Dirichlet dofs per element, or nullptr
  int npts;
  const double* pts;             // [npts][nv] barycentric, caller vertex order
  double *sig, *om;              // [ne][npts][d][d]
};

struct FacetSetupParams {
  Sizes s;
  int64_t nff;
  const int32_t* facet_el;
  const int32_t* facet_slot;
  const int32_t* elem_verts;
  const double* coords;
  const double* Ad;              // FP64 A^d, or nullptr: hi + lo in Adh, Adl
  const float *Adh, *Adl;
  const double *rcn, *rct;
  const int32_t* facet_out;      // 1: outlet facet (pi_0: no tangential rows in E)
  double* Dinv;
  float* Dinv32;
  double* DinvP;                 // upper triangles packed row by row (or nullptr)
  float* DinvP32;
  double* EF;
  float* EF32;
  int* status;
  // smoother 3: the l1 terms added to the diagonal of each facet block before
  // it is inverted ([free facet][n_fb], or nullptr), and the assembled
  // diagonal of A^d they are computed from
  const double* l1diag;
  double* addiag;
  const int32_t* elem_ff;
};

// One lattice block of a multigrid level (see MGBlock).
struct MGBlockDev {
  int n[3];
  int nc3[3];
  int prob, ffm;                  // ffm: faces whose vertices carry P1 dofs (outlets)
  int64_t voff, nvert, cvoff, nvert_c, nc, cmap_off, cinv_off;
};

// Loads a block descriptor (same address in every lane) and moves its fields
// to scalar registers, so that the index arithmetic on them stays scalar.
__device__ inline int uni32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
// A lattice vertex with coordinates c in a block of n intervals per axis carries
// P1 dofs when on every axis it is interior or lies on an outlet face (bit 2a
// of ffm: the face c_a = 0 is an outlet; bit 2a + 1: c_a = n_a); vertices on a
// Dirichlet face carry none.
__host__ __device__ inline bool lat_free(const int c[3], const int* n, int d, int ffm) {
  for (int a = 0; a < d; ++a) {
    if (c[a] < 0 || c[a] > n[a]) return false;
    if (c[a] == 0 && !((ffm >> (2 * a)) & 1)) return false;
    if (c[a] == n[a] && !((ffm >> (2 * a + 1)) & 1)) return false;
  }
  return true;
}

__device__ inline MGBlockDev load_block(const MGBlockDev* p) {
  MGBlockDev b = *p;
  for (int a = 0; a < 3; ++a) {
    b.n[a] = uni32(b.n[a]);
    b.nc3[a] = uni32(b.nc3[a]);
  }
  b.prob = uni32(b.prob);
  b.ffm = uni32(b.ffm);
  b.voff = uni64(b.voff);
  b.nvert = uni64(b.nvert);
  b.cvoff = uni64(b.cvoff);
  b.nvert_c = uni64(b.nvert_c);
  b.nc = uni64(b.nc);
  b.cmap_off = uni64(b.cmap_off);
  b.cinv_off = uni64(b.cinv_off);
  return b;
}

struct P1Params {
  int d;
  int nblk;                   // all blocks of the finest level
  const MGBlockDev* blk;
  int64_t maxv;
  const int32_t* vert_elem_off;
  const int32_t* vert_elem;
  const int32_t* elem_verts;
  const double* coords;
  const double* nu;
  double* A;
  int k;                      // order (outlet penalty nu C k^2 / h)
  double penalty;             // C
};

struct MGSetupParams {
  int d;
  int nblk, ncont;            // blocks of the level; the first ncont continue
  const MGBlockDev* blk;
  int64_t maxv, maxvc, maxnc;
  const double* A;            // this level's stencil
  double* Ac;                 // next level's stencil
  double* Dinv;
  float* Dinv32;
  const int32_t* cmap;
};

// Solve-phase constants.
struct SolveParams {
  Sizes s;
  int64_t ne, nff, off_f, off_p, ndof;
  const int32_t* elem_ff;
  const int32_t* facet_el;
  const int32_t* facet_slot;
  // [nff][4] per colour position: facet g, neighbours e1, e2 (-1: none) and
  // their local facet slots s1 | s2 << 8 (one 16-byte record)
  const int32_t* colour_desc;
  const double* detJ;
  const double* nu;
  const double* rBp;
  const double* rMpinv;
  // union of several problems: member of each element / free facet and a
  // per-member activity flag; work of inactive members is skipped.  active ==
  // nullptr: every member is active.
  const int32_t* elem_prob;
  const int32_t* facet_prob;
  const int32_t* active;
  // measurement: when set, the smoother kernel counts the facet blocks it
  // processes, spread over 256 counters 128 bytes apart (workgroup w adds to
  // counter w mod 256)
  unsigned long long* work_count;
  int has_outlet;  // some free facets are outlets with one neighbour
  // Dirichlet dofs per element ([ne][nd]): when set, gathers of facet values
  // take them for the element's Dirichlet facets (lifting and point values)
  const double* xD;
  // rows of A^d per thread in the operator apply (1, 2 or 4; 0: the largest
  // that n_d and the word size allow); every choice gives bitwise the same sums
  int apply_rpt;
};

__device__ inline bool elem_off(const SolveParams& P, int64_t e) {
  return P.active && !P.active[P.elem_prob[e]];
}
__device__ inline bool facet_off(const SolveParams& P, int64_t g) {
  return P.active && !P.active[P.facet_prob[g]];
}

// Full-system variant: overlapping blocks, one per facet of the mesh
// (Dirichlet facets included), holding the facet's free dofs and the bubbles
// of its neighbours; the velocity block A_T per element (reordered local
// order, FP64) and the bubble rows of the embedding E.
struct FullDev {
  int64_t nblk;
  int nbk;                        // block stride n_fb + 2 n_b
  const int32_t* blk_el;          // [nblk][2] neighbours (-1: none)
  const int32_t* blk_slot;        // [nblk][2] local facet index in the neighbour
  const int32_t* blk_g;           // [nblk] free facet id or -1
  const int32_t* colour_blocks;   // blocks sorted by colour
  const double* A;                // [ne][nA][nA]
  double* Binv;                   // [nblk][nbk][nbk]
  double* W;                      // [ne][(d+1)d][nA]  A_T E_T
  double* Eo;                     // [ne][n_b][(d+1)d] bubble rows of E_T
  const double* Eo_ref;           // [d+1][d][n_b]     lambda_v e_r on the reference element
};

template <typename R>
struct OpPtrs {
  const R *Ad, *H, *Aoo, *Aooinv, *Dinv, *EF, *W;
  // split storage of A^d, H, A_oo (R = double with Ad == nullptr)
  const float *hAd, *lAd, *hH, *lH, *hAoo, *lAoo;
  // D_F^{-1} (symmetric) as packed upper triangles: entry (i, j), i <= j, at
  // i n_fb - i (i - 1) / 2 + j - i of the facet's n_fb (n_fb + 1) / 2 words
  const R* DinvP;
};

// Matrix entry accessors: plain arrays, or FP64 values kept as FP32 hi + lo.
template <typename R>
struct MatP {
  const R* p;
  __device__ R operator()(size_t i) const { return p[i]; }
};
struct MatHL {
  const float* h;
  const float* l;
  __device__ double operator()(size_t i) const { return (double)h[i] + (double)l[i]; }
};

struct MGLevelDev {
  int nblk, ncont;            // blocks of the level; the first ncont continue
  const MGBlockDev* blk;
  int64_t maxv, maxvc, maxnc;
  const void* A;      // stencil (R)
  const void* Dinv;   // (R)
  void *x, *b, *r;    // lattice vectors (R)
  const int32_t* active;  // per-member activity (nullptr: all active)
};

// ---------------------------------------------------------------------------
// Batched solves: the global vectors of a union are cut into tiles that never
// straddle two member problems (per member: its bubble, facet and pressure
// sections, in that order), so per-member reductions are sums over the
// member's own tiles in a fixed order, independent of the other members.
// ---------------------------------------------------------------------------
struct SegTile {
  int32_t prob, len;
  int64_t start;
};

// Per-member MINRES scalars, stored field-major: st[field * nprob + member].
enum {
  ST_BETA = 0, ST_OLDB, ST_DBAR, ST_EPS, ST_PHIBAR, ST_CS, ST_SN, ST_BETA1, ST_STOP, ST_ALPHA, ST_BB,
  ST_CW0, ST_CW1, ST_CW2, ST_PHI, ST_REL, ST_TOL, ST_ABS, ST_SB1, ST_RN, ST_NFIELD
};

struct SegDev {
  int nprob;
  int64_t ntiles;
  const SegTile* tiles;
  const int32_t* tile_off;   // [nprob+1]
  double* partial;           // [ntiles]
  double* st;                // [ST_NFIELD][nprob]
  int32_t* active;           // mask used by this operation
  int32_t* its;              // iterations of the current MINRES
  int32_t* status;           // mcs_status per member
  int32_t* done;             // set when a member leaves the iteration
  int maxit;
};

}  // namespace mcs
