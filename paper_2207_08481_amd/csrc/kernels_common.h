// Kernel parameter blocks shared by the setup and solve kernels.
#pragma once
#include "mcs_internal.h"

namespace mcs {

constexpr int MAXND = 256;   // max A^d size (k = 5, 3D: 204)
constexpr int MAXNB = 96;    // max bubbles (84)
constexpr int MAXNP = 40;    // max pressure dofs (35)
constexpr int MAXNFB = 64;   // max facet block (51)

struct CondParams {
  Sizes s;
  int64_t ne;
  int64_t slot_doubles;
  const int32_t* elem_verts;
  const double* coords;
  const double* nu;
  const double *rV, *rBf, *rU, *rL, *rD;
  double facet_measure[4];
  double* scratch;
  double* detJ;
  double *Ad, *H, *Aoo, *Aooinv;
  float *Ad32, *H32, *Aoo32, *Aooinv32;
  int* status;
};

struct FacetSetupParams {
  Sizes s;
  int64_t nff;
  const int32_t* facet_el;
  const int32_t* facet_slot;
  const int32_t* elem_verts;
  const double* coords;
  const double* Ad;
  const double *rcn, *rct;
  double* Dinv;
  float* Dinv32;
  double* EF;
  float* EF32;
  int* status;
};

struct P1Params {
  int d;
  int n[3];
  int64_t nvert;
  const int32_t* vert_elem_off;
  const int32_t* vert_elem;
  const int32_t* elem_verts;
  const double* coords;
  const double* nu;
  double* A;
};

struct MGSetupParams {
  int d;
  int n[3];       // fine intervals
  int nc[3];      // coarse intervals
  int64_t nvert, nvert_c, ncd;
  const double* A;
  double* Ac;
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
  const int32_t* colour_facets;
  const double* detJ;
  const double* nu;
  const double* rBp;
  const double* rMpinv;
};

template <typename R>
struct OpPtrs {
  const R *Ad, *H, *Aoo, *Aooinv, *Dinv, *EF, *W;
};

struct MGLevelDev {
  int n[3];
  int64_t nvert;
  const void* A;      // stencil (R)
  const void* Dinv;   // (R)
  void *x, *b, *r;    // lattice vectors (R)
};

}  // namespace mcs
