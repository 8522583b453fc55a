// Setup kernels: element matrices and static condensation (Sec. 4.2,
// eq. bigfemSPmat, eq. factorSsigma), facet smoother blocks (Theorem
// aux_pc_schur), embedding blocks E^d (eq. defE, eq. defED) and the P1
// multigrid hierarchy for A-bar (eq. defAhat).
//
// Condensation I is computed in a reduced form that is algebraically equal to
// A = A^div - B_sigma M^{-1} B_sigma^T: the stress space is described by an
// L2-orthonormal scalar basis psi_a times an orthonormal basis D_m of
// trace-free matrices, the symmetry multiplier omega is eliminated by keeping
// only the top-degree part of the skew components (sigma is orthogonal to
// P^{k-1}(T, K) exactly when its skew part lies in P^k minus P^{k-1}), and the
// nt-trace degree condition of Sigma_h is imposed through its constraint
// matrix Lambda.  With the mass matrix (|T|/nu) I this gives
//     A = A^div + (nu/|T|) G (I - Q^T Q) G^T,
// G[i, (a,m)] = b(psi_a D_m, phi_i), Q an orthonormal basis of the rows of
// Lambda (obtained by two Cholesky-QR passes).
#include "kernels_common.h"
#include "launch.h"

namespace mcs {

// --------------------------------------------------------------------------
// 64x64 output tiles of dense products on the FP64 matrix cores, 256 threads:
// wave w owns the 32x32 quarter (w / 2, w % 2) as 2x2 blocks of the 16x16x4
// FP64 matrix instruction; K panels of 16 are staged in LDS as [k][64].
// Operand lanes: A(i, k) in lane i + 16 k, B^T(k, j) in lane j + 16 k;
// result register r of lane l holds C(l / 16 + 4 r, l % 16) of a block.
// acc[q], q = 8 bi + 4 bj + r, is C[m0 + tile_row(q)][n0 + tile_col(q)].
// --------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline int tile_row(int q) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w >> 1) * 32 + (q >> 3) * 16 + (l >> 4) + 4 * (q & 3);
}
__device__ inline int tile_col(int q) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w & 1) * 32 + ((q >> 2) & 1) * 16 + (l & 15);
}

// c += la-panel x lb-panel^T for this wave's quarter (one 16-deep panel).
__device__ inline void tile_panel_mfma(const double* la, const double* lb, dbl4 c[2][2]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rb = (w >> 1) * 32 + (l & 15), cb = (w & 1) * 32 + (l & 15);
#pragma unroll
  for (int k4 = 0; k4 < 16; k4 += 4) {
    const int kk = (k4 + (l >> 4)) * 64;
    const double a0 = la[kk + rb], a1 = la[kk + rb + 16];
    const double b0 = lb[kk + cb], b1 = lb[kk + cb + 16];
    c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c[0][0], 0, 0, 0);
    c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c[0][1], 0, 0, 0);
    c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c[1][0], 0, 0, 0);
    c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c[1][1], 0, 0, 0);
  }
}

__device__ inline void tile_store(const dbl4 c[2][2], double acc[16]) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bi * 8 + bj * 4 + r] = c[bi][bj][r];
}

// C = A B^T (A: M x K, B: N x K, row-major): the tile at (m0, n0).
__device__ void tile_nt(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                        int m0, int n0, int M, int N, int K, double acc[16], double* lds) {
  double* la = lds;            // [16][64]
  double* lb = lds + 16 * 64;  // [16][64]
  const int tid = threadIdx.x;
  dbl4 c[2][2];
  for (int bi = 0; bi < 2; ++bi)
    for (int bj = 0; bj < 2; ++bj) c[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int idx = tid; idx < 1024; idx += 256) {
      int r = idx >> 4, kk = idx & 15;
      int gm = m0 + r, gn = n0 + r, gk = k0 + kk;
      la[kk * 64 + r] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.0;
      lb[kk * 64 + r] = (gn < N && gk < K) ? B[(size_t)gn * ldb + gk] : 0.0;
    }
    __syncthreads();
    tile_panel_mfma(la, lb, c);
    __syncthreads();
  }
  tile_store(c, acc);
}

// C = A B for row-major A (M x K, lda) and B (K x N, ldb): the tile at (m0, n0).
__device__ void tile_nn(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                        int m0, int n0, int M, int N, int K, double acc[16], double* lds) {
  double* la = lds;            // [16][64]
  double* lb = lds + 16 * 64;  // [16][64]
  const int tid = threadIdx.x;
  dbl4 c[2][2];
  for (int bi = 0; bi < 2; ++bi)
    for (int bj = 0; bj < 2; ++bj) c[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int idx = tid; idx < 1024; idx += 256) {
      int r = idx >> 4, kk = idx & 15;
      int gm = m0 + r, gk = k0 + kk;
      la[kk * 64 + r] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.0;
      int kb = idx >> 6, cc = idx & 63;
      int gkb = k0 + kb, gn = n0 + cc;
      lb[kb * 64 + cc] = (gkb < K && gn < N) ? B[(size_t)gkb * ldb + gn] : 0.0;
    }
    __syncthreads();
    tile_panel_mfma(la, lb, c);
    __syncthreads();
  }
  tile_store(c, acc);
}

// In-place Cholesky (lower) of an n x n row-major SPD matrix in memory
// visible to the block; returns false on breakdown.  Upper part zeroed.
__device__ bool block_cholesky(double* S, int n, int ld) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double v = S[j * ld + j];
      if (!(v > 0.0)) {
        bad = 1;
        v = 1.0;
      }
      S[j * ld + j] = sqrt(v);
    }
    __syncthreads();
    double piv = S[j * ld + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) S[i * ld + j] /= piv;
    __syncthreads();
    int m = n - j - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      int i = j + 1 + idx / m, c = j + 1 + idx % m;
      if (c <= i) S[i * ld + c] -= S[i * ld + j] * S[c * ld + j];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    int i = idx / n, c = idx % n;
    if (c > i) S[i * ld + c] = 0.0;
  }
  __syncthreads();
  return bad == 0;
}

// X <- L^{-1} X for lower-triangular L (n x n) and X (n x ncol), column parallel.
__device__ void block_trsm_lower(const double* L, int ldl, double* X, int ldx, int n, int ncol) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      double t = X[i * ldx + c];
      for (int p = 0; p < i; ++p) t -= L[i * ldl + p] * X[p * ldx + c];
      X[i * ldx + c] = t / L[i * ldl + i];
    }
  }
  __syncthreads();
}

// Inverse of an SPD matrix given its Cholesky factor L (in S, lower):
// out = L^{-T} L^{-1}.  W is n x n scratch.
__device__ void block_spd_inverse(const double* L, int n, double* W, double* out) {
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) W[idx] = ((idx / n) == (idx % n)) ? 1.0 : 0.0;
  __syncthreads();
  block_trsm_lower(L, n, W, n, n, n);   // W = L^{-1}
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    int i = idx / n, j = idx % n;
    int p0 = i > j ? i : j;
    double t = 0.0;
    for (int p = p0; p < n; ++p) t += W[p * n + i] * W[p * n + j];
    out[idx] = t;
  }
  __syncthreads();
}

// Orthonormal trace-free basis (Frobenius): symmetric part, then skew part.
__device__ void dm_basis(int d, int m, double D[3][3]) {
  const double r2 = 0.70710678118654752440, r6 = 0.40824829046386301637;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D[i][j] = 0.0;
  if (d == 2) {
    if (m == 0) { D[0][1] = r2; D[1][0] = r2; }
    else if (m == 1) { D[0][0] = r2; D[1][1] = -r2; }
    else { D[0][1] = r2; D[1][0] = -r2; }
  } else {
    switch (m) {
      case 0: D[0][1] = r2; D[1][0] = r2; break;
      case 1: D[0][2] = r2; D[2][0] = r2; break;
      case 2: D[1][2] = r2; D[2][1] = r2; break;
      case 3: D[0][0] = r2; D[1][1] = -r2; break;
      case 4: D[0][0] = r6; D[1][1] = r6; D[2][2] = -2.0 * r6; break;
      case 5: D[0][1] = r2; D[1][0] = -r2; break;
      case 6: D[0][2] = r2; D[2][0] = -r2; break;
      default: D[1][2] = r2; D[2][1] = -r2; break;
    }
  }
}

struct ElemGeo {
  double J[3][3], Ji[3][3], det, vol;
  double X[4][3];
  double n[4][3], area[4], t[4][2][3], gl[4][3];
};

__device__ void element_geometry(const CondParams& P, int64_t e, ElemGeo& g) {
  const int d = P.s.d, nv = d + 1;
  for (int j = 0; j < nv; ++j) {
    int v = P.elem_verts[e * nv + j];
    for (int r = 0; r < 3; ++r) g.X[j][r] = r < d ? P.coords[(size_t)v * d + r] : 0.0;
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) g.J[r][c] = (r < d && c < d) ? g.X[c + 1][r] - g.X[0][r] : (r == c ? 1.0 : 0.0);
  double (&J)[3][3] = g.J;
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  g.det = det;
  g.Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  g.Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  g.Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  g.Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  g.Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  g.Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  g.Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  g.Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  g.Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  g.vol = fabs(det) / (d == 2 ? 2.0 : 6.0);
  for (int r = 0; r < 3; ++r) {
    g.gl[0][r] = 0.0;
    for (int j = 1; j < nv; ++j) {
      g.gl[j][r] = r < d ? g.Ji[j - 1][r] : 0.0;
      g.gl[0][r] -= g.gl[j][r];
    }
  }
  for (int f = 0; f < nv; ++f) {
    double nn = 0.0;
    for (int r = 0; r < d; ++r) nn += g.gl[f][r] * g.gl[f][r];
    nn = sqrt(nn);
    for (int r = 0; r < 3; ++r) g.n[f][r] = r < d ? -g.gl[f][r] / nn : 0.0;
    g.area[f] = d * g.vol * nn;
    int fv[3], c = 0;
    for (int j = 0; j < nv; ++j)
      if (j != f) fv[c++] = j;
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 3; ++r) g.t[f][b][r] = (b < d - 1) ? g.X[fv[b + 1]][r] - g.X[fv[0]][r] : 0.0;
  }
}

// --------------------------------------------------------------------------
// Pieces shared by the condensation and the stress recovery.
// --------------------------------------------------------------------------
// Geometry of element e and the coefficient tables of the stress basis:
// sEm[m] = J^T D_m J^{-T}; sW[f][m] = (|F_f| / |F^_f|) J^T (tangential part of
// D_m n_f); sTd[f][b][m] = t_b . D_m n_f.  Block-wide; ends synchronised.
__device__ __forceinline__ void stress_tables(const CondParams& P, int64_t e, ElemGeo& g, double (*sEm)[3][3],
                                              double (*sW)[8][3], double (*sTd)[2][8]) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1, nD = s.nsym + s.nskew;
  const int tid = threadIdx.x;
  if (tid == 0) element_geometry(P, e, g);
  __syncthreads();
  for (int idx = tid; idx < nD * nv; idx += blockDim.x) {
    int m = idx % nD, f = idx / nD;
    double D[3][3];
    dm_basis(d, m, D);
    if (f == 0) {  // Em = J^T D_m J^{-T}
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
          double t = 0.0;
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) t += g.J[a][r] * D[a][b] * g.Ji[c][b];
          sEm[m][r][c] = t;
        }
    }
    double Dn[3] = {0, 0, 0}, nDn = 0.0;
    for (int a = 0; a < d; ++a) {
      for (int b = 0; b < d; ++b) Dn[a] += D[a][b] * g.n[f][b];
      nDn += g.n[f][a] * Dn[a];
    }
    double Pt[3];
    for (int a = 0; a < d; ++a) Pt[a] = Dn[a] - g.n[f][a] * nDn;
    double sc = g.area[f] / P.facet_measure[f];
    for (int r = 0; r < d; ++r) {
      double t = 0.0;
      for (int a = 0; a < d; ++a) t += g.J[a][r] * Pt[a];
      sW[f][m][r] = sc * t;
    }
    for (int b = 0; b < d - 1; ++b) {
      double t = 0.0;
      for (int a = 0; a < d; ++a) t += g.t[f][b][a] * Dn[a];
      sTd[f][b][m] = t;
    }
  }
  __syncthreads();
}

// Column c of the reduced stress space -> (trace-free basis index m, scalar
// index a): every psi_a for the symmetric D_m, only the top-degree psi_a for
// the skew D_m (a >= sklo = n_{k-1}); for k = 1 omega is not condensed and
// the skew D_m keep every psi_a (sklo = 0).
__device__ __forceinline__ void sig_col(const Sizes& s, int c, int& m, int& a) {
  const int ntop = s.ns - s.sklo;
  if (c < s.nsym * s.ns) {
    m = c / s.ns;
    a = c % s.ns;
  } else {
    const int cc = c - s.nsym * s.ns;
    m = s.nsym + cc / ntop;
    a = s.sklo + cc % ntop;
  }
}

// k = 1 (Sec. 7): omega in the lowest-order Raviart-Thomas space, one flux
// dof per facet f w.r.t. the facet's global normal (sorted vertices:
// (x_b - x_a) x (x_c - x_a)): psi_f = s_f (x - x_f) / (d |T|), s_f = +-1 its
// orientation against the outward normal, div psi_f = s_f / |T|.
__device__ __forceinline__ double rt_sign(const ElemGeo& g, int f) {
  const double* t0 = g.t[f][0];
  const double* t1 = g.t[f][1];
  const double c0 = t0[1] * t1[2] - t0[2] * t1[1], c1 = t0[2] * t1[0] - t0[0] * t1[2],
               c2 = t0[0] * t1[1] - t0[1] * t1[0];
  return c0 * g.n[f][0] + c1 * g.n[f][1] + c2 * g.n[f][2] > 0.0 ? 1.0 : -1.0;
}

// G[i, (m, a)] = b(psi_a D_m, phi_i) for the local velocity row i (order:
// bubbles, then per facet its normal functions and tangential functions).
__device__ __forceinline__ double g_entry(const CondParams& P, const ElemGeo& g, const double (*sEm)[3][3],
                                          const double (*sW)[8][3], const double (*sTd)[2][8], int i, int m, int a,
                                          double adet, double idet) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1;
  int iu = -1, f = 0, q = 0;
  double sc = 1.0;
  if (i < s.nb) iu = i;
  else {
    f = (i - s.nb) / s.nfb;
    q = (i - s.nb) % s.nfb;
    if (q < s.nF) { iu = s.nb + f * s.nF + q; sc = idet; }
  }
  if (q >= s.nF + s.nh) {
    // omega row (k = 1): int_T psi_a D_m : kappa(psi_f), kappa(w) the skew
    // matrix with kappa(curl u) = skew(grad u), i.e. (1/2) [w]_x.  With
    // x - x_f = sum_j lambda_j (x_j - x_f) and |T| = |det J| |T^|:
    //   s_f / (d |T^|) sum_j (D_m : kappa(x_j - x_f)) int_T^ psi_a lambda_j
    double D[3][3];
    dm_basis(d, m, D);
    double t = 0.0;
    for (int j = 0; j < nv; ++j) {
      if (j == f) continue;
      double w[3];
      for (int r = 0; r < 3; ++r) w[r] = g.X[j][r] - g.X[f][r];
      // D : (1/2)[w]_x, [w]_x = [[0,-w2,w1],[w2,0,-w0],[-w1,w0,0]]
      const double dk = 0.5 * (-D[0][1] * w[2] + D[0][2] * w[1] + D[1][0] * w[2] - D[1][2] * w[0] -
                               D[2][0] * w[1] + D[2][1] * w[0]);
      t += dk * P.rLam[(size_t)a * nv + j];
    }
    return rt_sign(g, f) * t * 2.0;   // (d - 1)! = 2: k = 1 is three-dimensional
  }
  if (iu >= 0) {
    double t = 0.0;
    const double* Vp = P.rV + ((size_t)iu * s.ns + a) * d * d;
    for (int r = 0; r < d; ++r)
      for (int c2 = 0; c2 < d; ++c2) t += sEm[m][r][c2] * Vp[r * d + c2];
    t *= -adet;
    for (int ff = 0; ff < nv; ++ff) {
      const double* Bp = P.rBf + (((size_t)ff * s.nu + iu) * s.ns + a) * d;
      for (int r = 0; r < d; ++r) t += sW[ff][m][r] * Bp[r];
    }
    return sc * t;
  }
  const int j = q - s.nF, b = j / s.nFkm1, gm = j % s.nFkm1;
  return -(g.area[f] / P.facet_measure[f]) * sTd[f][b][m] * P.rU[((size_t)f * s.nFkm1 + gm) * s.ns + a];
}

// Lambda (the top-degree nt-trace moments of the reduced stress columns),
// made row-orthonormal in place by two Cholesky-QR passes (Lm: nlam x nsig,
// sS: 48 x 48 LDS).  Returns false on a Cholesky breakdown.
__device__ __forceinline__ bool lambda_q(const CondParams& P, const double (*sTd)[2][8], double* Lm, double* sS) {
  const Sizes s = P.s;
  const int d = s.d, nq = s.nFk - s.nFkm1;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < s.nlam * s.nsig; idx += blockDim.x) {
    int l = idx / s.nsig, m, a;
    sig_col(s, idx % s.nsig, m, a);
    int qq = l % nq, fb = l / nq, f = fb / (d - 1), b = fb % (d - 1);
    Lm[idx] = sTd[f][b][m] * P.rL[((size_t)f * nq + qq) * s.ns + a];
  }
  __syncthreads();
  bool ok = true;
  for (int pass = 0; pass < 2; ++pass) {
    for (int idx = tid; idx < s.nlam * s.nlam; idx += blockDim.x) {
      int i = idx / s.nlam, j = idx % s.nlam;
      double t = 0.0;
      for (int c = 0; c < s.nsig; ++c) t += Lm[i * s.nsig + c] * Lm[j * s.nsig + c];
      sS[i * 48 + j] = t;
    }
    __syncthreads();
    ok = block_cholesky(sS, s.nlam, 48) && ok;
    block_trsm_lower(sS, 48, Lm, s.nsig, s.nlam, s.nsig);
  }
  return ok;
}

__global__ void __launch_bounds__(256) k_condense(CondParams P) {
  const Sizes s = P.s;
  const int d = s.d;
  const int tid = threadIdx.x;
  __shared__ ElemGeo g;
  __shared__ double sEm[8][3][3];
  __shared__ double sW[4][8][3];
  __shared__ double sTd[4][2][8];
  __shared__ double sS[48 * 48];
  __shared__ double lds[2 * 16 * 64];
  double* scr = P.scratch + (size_t)blockIdx.x * P.slot_doubles;
  double* G = scr;                                   // nA x nsig
  double* Lm = G + (size_t)s.nA * s.nsig;            // nlam x nsig
  double* Y = Lm + (size_t)s.nlam * s.nsig;          // nA x nlam
  double* A = Y + (size_t)s.nA * s.nlam;             // nA x nA
  double* Ai = A + (size_t)s.nA * s.nA;              // nb x nb
  double* Wk = Ai + (size_t)s.nb * s.nb;             // nb x nb

  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    stress_tables(P, e, g, sEm, sW, sTd);
    const double adet = fabs(g.det), idet = 1.0 / g.det;
    // G (reordered local rows)
    for (int64_t idx = tid; idx < (int64_t)s.nA * s.nsig; idx += blockDim.x) {
      int i = (int)(idx / s.nsig), m, a;
      sig_col(s, (int)(idx % s.nsig), m, a);
      G[idx] = g_entry(P, g, sEm, sW, sTd, i, m, a, adet, idet);
    }
    bool ok = lambda_q(P, sTd, Lm, sS);
    // Y = G Q^T
    for (int n0 = 0; n0 < s.nlam; n0 += 64)
      for (int m0 = 0; m0 < s.nA; m0 += 64) {
        double acc[16];
        tile_nt(G, s.nsig, Lm, s.nsig, m0, n0, s.nA, s.nlam, s.nsig, acc, lds);
        for (int q = 0; q < 16; ++q) {
          int r = m0 + tile_row(q), c = n0 + tile_col(q);
          if (r < s.nA && c < s.nlam) Y[r * s.nlam + c] = acc[q];
        }
      }
    __syncthreads();
    // R = G (I - Q^T Q) = G - Y Q  (in place of G): the sigma columns with the
    // nt-constraint directions projected out
    for (int m0 = 0; m0 < s.nA; m0 += 64)
      for (int n0 = 0; n0 < s.nsig; n0 += 64) {
        double acc[16];
        tile_nn(Y, s.nlam, Lm, s.nsig, m0, n0, s.nA, s.nsig, s.nlam, acc, lds);
        for (int q = 0; q < 16; ++q) {
          int r = m0 + tile_row(q), c = n0 + tile_col(q);
          if (r < s.nA && c < s.nsig) G[(size_t)r * s.nsig + c] -= acc[q];
        }
      }
    __syncthreads();
    // A = A^div + (nu/|T|) R R^T   (= G (I - Q^T Q) G^T without the
    // cancellation of two large Gram matrices)
    const double nuT = P.nu[e];
    const double cf = nuT / g.vol;
    for (int m0 = 0; m0 < s.nA; m0 += 64)
      for (int n0 = m0; n0 < s.nA; n0 += 64) {
        double acc[16];
        tile_nt(G, s.nsig, G, s.nsig, m0, n0, s.nA, s.nA, s.nsig, acc, lds);
        for (int q = 0; q < 16; ++q) {
          int r = m0 + tile_row(q), c = n0 + tile_col(q);
          // upper triangle only (in a diagonal block the (c, r) thread would
          // write the mirrored pair too): one writer per entry pair
          if (r < s.nA && c < s.nA && r <= c) {
            double v = cf * acc[q];
            // A^div on velocity rows
            int ir = -1, ic = -1;
            double sr = 1.0, sc2 = 1.0;
            if (r < s.nb) ir = r;
            else { int f = (r - s.nb) / s.nfb, t = (r - s.nb) % s.nfb; if (t < s.nF) { ir = s.nb + f * s.nF + t; sr = idet; } }
            if (c < s.nb) ic = c;
            else { int f = (c - s.nb) / s.nfb, t = (c - s.nb) % s.nfb; if (t < s.nF) { ic = s.nb + f * s.nF + t; sc2 = idet; } }
            if (ir >= 0 && ic >= 0) v += (nuT / d) * sr * sc2 * adet * P.rD[(size_t)ir * s.nu + ic];
            if (s.nw) {
              // k = 1: nu |T|^(2/3) (div omega, div eta)_T on the omega rows,
              // div psi_f = s_f / |T|
              const int tr = (r - s.nb) % s.nfb, tc = (c - s.nb) % s.nfb;
              if (r >= s.nb && c >= s.nb && tr == s.nF + s.nh && tc == s.nF + s.nh) {
                const double c23 = cbrt(g.vol);
                v += nuT * c23 * c23 * rt_sign(g, (r - s.nb) / s.nfb) * rt_sign(g, (c - s.nb) / s.nfb) / g.vol;
              }
            }
            A[(size_t)r * s.nA + c] = v;
            A[(size_t)c * s.nA + r] = v;
          }
        }
      }
    __syncthreads();
    // tangential dofs of an outlet facet are fixed to zero: identity rows and
    // columns, so that they decouple before the bubbles are condensed (k = 1:
    // the omega flux stays free there, W_h vanishes on Gamma_D only, Sec. 7)
    if (P.facet_out) {
      const int nv = d + 1;
      auto pinned = [&](int r) {
        if (r < s.nb) return false;
        const int f = (r - s.nb) / s.nfb, q = (r - s.nb) % s.nfb;
        const int gf = P.elem_ff[e * nv + f];
        return q >= s.nF && q < s.nF + s.nh && gf >= 0 && P.facet_out[gf] != 0;
      };
      for (int idx = tid; idx < s.nA * s.nA; idx += blockDim.x) {
        const int r = idx / s.nA, c = idx % s.nA;
        if (pinned(r) || pinned(c)) A[idx] = r == c ? 1.0 : 0.0;
      }
      __syncthreads();
    }
    if (P.Afull)
      for (int idx = tid; idx < s.nA * s.nA; idx += blockDim.x) P.Afull[(size_t)e * s.nA * s.nA + idx] = A[idx];
    // condensation II: Aoo = A[0:nb,0:nb]
    const int nb = s.nb, nd = s.nd;
    for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
      int i = idx / nb, j = idx % nb;
      double v = A[(size_t)i * s.nA + j];
      Wk[idx] = v;
      const float hv = (float)v;
      if (P.Aoo) P.Aoo[(size_t)e * nb * nb + idx] = v;
      P.Aoo32[(size_t)e * nb * nb + idx] = hv;
      if (P.Aool) P.Aool[(size_t)e * nb * nb + idx] = (float)(v - (double)hv);
    }
    __syncthreads();
    ok = block_cholesky(Wk, nb, nb) && ok;
    for (int idx = tid; idx < nb * nb; idx += blockDim.x) Ai[idx] = ((idx / nb) == (idx % nb)) ? 1.0 : 0.0;
    __syncthreads();
    block_trsm_lower(Wk, nb, Ai, nb, nb, nb);  // Ai = L^{-1}
    for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
      int i = idx / nb, j = idx % nb;
      int p0 = i > j ? i : j;
      double t = 0.0;
      for (int p = p0; p < nb; ++p) t += Ai[p * nb + i] * Ai[p * nb + j];
      Wk[idx] = t;  // Wk = Aoo^{-1}
    }
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
      if (P.Aooinv) P.Aooinv[(size_t)e * nb * nb + idx] = Wk[idx];
      P.Aooinv32[(size_t)e * nb * nb + idx] = (float)Wk[idx];
    }
    // Ht[n][m] = sum_k A[nb+n][k] Aooinv[m][k]   (nd x nb), kept in the slot
    // scratch (the sigma columns G are no longer needed)
    double* Ht = G;
    for (int m0 = 0; m0 < nd; m0 += 64)
      for (int n0 = 0; n0 < nb; n0 += 64) {
        double acc[16];
        tile_nt(A + (size_t)nb * s.nA, s.nA, Wk, nb, m0, n0, nd, nb, nb, acc, lds);
        for (int q = 0; q < 16; ++q) {
          int r = m0 + tile_row(q), c = n0 + tile_col(q);
          if (r < nd && c < nb) {
            double v = acc[q];
            Ht[(size_t)r * nb + c] = v;
            const size_t hi = (size_t)e * nb * nd + (size_t)c * nd + r;
            const float hv = (float)v;
            if (P.H) P.H[hi] = v;
            P.H32[hi] = hv;
            if (P.Hl) P.Hl[hi] = (float)(v - (double)hv);
          }
        }
      }
    __syncthreads();
    // Ad = A_dd - A_do Ht^T   (in the FP64 array, or the slot's FP64 buffer)
    double* Ade = P.Ad ? P.Ad + (size_t)e * nd * nd : P.adtmp + (size_t)blockIdx.x * P.adtmp_stride;
    for (int m0 = 0; m0 < nd; m0 += 64)
      for (int n0 = 0; n0 < nd; n0 += 64) {
        double acc[16];
        tile_nt(A + (size_t)nb * s.nA, s.nA, Ht, nb, m0, n0, nd, nd, nb, acc, lds);
        for (int q = 0; q < 16; ++q) {
          int r = m0 + tile_row(q), c = n0 + tile_col(q);
          if (r < nd && c < nd) {
            double v = A[(size_t)(nb + r) * s.nA + nb + c] - acc[q];
            Ade[(size_t)r * nd + c] = v;
          }
        }
      }
    __syncthreads();
    // symmetrise Ad exactly and write the FP32 copy (and the low parts)
    for (int idx = tid; idx < nd * nd; idx += blockDim.x) {
      int r = idx / nd, c = idx % nd;
      if (c < r) continue;
      double v = 0.5 * (Ade[(size_t)r * nd + c] + Ade[(size_t)c * nd + r]);
      Ade[(size_t)r * nd + c] = v;
      Ade[(size_t)c * nd + r] = v;
      const float hv = (float)v;
      P.Ad32[(size_t)e * nd * nd + (size_t)r * nd + c] = hv;
      P.Ad32[(size_t)e * nd * nd + (size_t)c * nd + r] = hv;
      if (P.Adl) {
        const float lv = (float)(v - (double)hv);
        P.Adl[(size_t)e * nd * nd + (size_t)r * nd + c] = lv;
        P.Adl[(size_t)e * nd * nd + (size_t)c * nd + r] = lv;
      }
    }
    if (tid == 0) {
      P.detJ[e] = g.det;
      if (!ok) atomicOr(P.status, 1);
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// Facet smoother blocks D_F = sum_{T ni F} (A^d_T)_{FF} and their inverses,
// and the embedding blocks E_F (facet rows of E u = (u, u_t), eq. defE):
//   normal rows:     |F| (e_c . n_F) * coefficient of lambda_v in the degree-k
//                    facet Bernstein basis (facet functions have normal trace
//                    lambda^beta / |F|);
//   tangential rows: coefficient of lambda_v in degree k-1 times the
//                    coordinates of P_t e_c in the tangent basis t_b.
// --------------------------------------------------------------------------
// l1 terms of the facet block l1-Jacobi smoother (smoother 3): for facet dof
// i = (g, q), l_i = sum over the free dofs j of the other facets of its
// neighbours of |a_ij| sqrt(a_ii / a_jj), a the assembled A^d (two facets
// share at most one element, so a_ij is that element's entry).  Pass 0 forms
// the assembled diagonal, pass 1 the sums.
__device__ inline double ad_entry(const FacetSetupParams& P, size_t i) {
  return P.Ad ? P.Ad[i] : (double)P.Adh[i] + (double)P.Adl[i];
}
__global__ void k_l1_terms(FacetSetupParams P, int pass, double* __restrict__ out) {
  const Sizes s = P.s;
  const int nfb = s.nfb, nd = s.nd, nv = s.d + 1;
  const int64_t n = P.nff * nfb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = idx / nfb;
    const int q = (int)(idx % nfb);
    double t = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int64_t e = P.facet_el[2 * g + side];
      if (e < 0) continue;
      const int sl = P.facet_slot[2 * g + side];
      const size_t row = (size_t)e * nd * nd + (size_t)(sl * nfb + q) * nd;
      if (pass == 0) {
        t += ad_entry(P, row + sl * nfb + q);
        continue;
      }
      const double si = sqrt(P.addiag[idx]);
      for (int h = 0; h < nv; ++h) {
        if (h == sl) continue;
        const int G = P.elem_ff[e * nv + h];
        if (G < 0) continue;
        for (int qq = 0; qq < nfb; ++qq)
          t += fabs(ad_entry(P, row + h * nfb + qq)) * si / sqrt(P.addiag[(int64_t)G * nfb + qq]);
      }
    }
    out[idx] = t;
  }
}

void launch_l1_terms(hipStream_t st, const FacetSetupParams& P, double* diag, double* l1) {
  const int64_t n = P.nff * P.s.nfb;
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 20))), b(256);
  FacetSetupParams Q = P;
  hipLaunchKernelGGL(k_l1_terms, g, b, 0, st, Q, 0, diag);
  Q.addiag = diag;
  hipLaunchKernelGGL(k_l1_terms, g, b, 0, st, Q, 1, l1);
}

__global__ void __launch_bounds__(256) k_facet_setup(FacetSetupParams P) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1, nfb = s.nfb, nd = s.nd;
  constexpr int FLD = 52;  // leading dimension of the facet block (n_fb <= 51)
  __shared__ double S[FLD * FLD];
  __shared__ double W[FLD * FLD];
  __shared__ double X[3][3];
  __shared__ double geo[16];
  for (int64_t g = blockIdx.x; g < P.nff; g += gridDim.x) {
    for (int idx = threadIdx.x; idx < nfb * nfb; idx += blockDim.x) {
      int i = idx / nfb, j = idx % nfb;
      double t = 0.0;
      for (int side = 0; side < 2; ++side) {
        int64_t e = P.facet_el[2 * g + side];
        if (e < 0) continue;   // outlet facet: one neighbour
        int sl = P.facet_slot[2 * g + side];
        const size_t ai = (size_t)e * nd * nd + (size_t)(sl * nfb + i) * nd + sl * nfb + j;
        t += P.Ad ? P.Ad[ai] : (double)P.Adh[ai] + (double)P.Adl[ai];
      }
      S[i * FLD + j] = t + (i == j && P.l1diag ? P.l1diag[g * nfb + i] : 0.0);
    }
    __syncthreads();
    bool ok = block_cholesky(S, nfb, FLD);
    for (int idx = threadIdx.x; idx < nfb * nfb; idx += blockDim.x) W[(idx / nfb) * FLD + idx % nfb] = ((idx / nfb) == (idx % nfb)) ? 1.0 : 0.0;
    __syncthreads();
    block_trsm_lower(S, FLD, W, FLD, nfb, nfb);
    for (int idx = threadIdx.x; idx < nfb * nfb; idx += blockDim.x) {
      int i = idx / nfb, j = idx % nfb;
      int p0 = i > j ? i : j;
      double t = 0.0;
      for (int p = p0; p < nfb; ++p) t += W[p * FLD + i] * W[p * FLD + j];
      if (P.Dinv) P.Dinv[(size_t)g * nfb * nfb + idx] = t;
      P.Dinv32[(size_t)g * nfb * nfb + idx] = (float)t;
      if (i <= j) {   // the same sum for (i, j) and (j, i): the matrix is exactly symmetric
        const size_t pk = (size_t)g * (nfb * (nfb + 1) / 2) + i * nfb - i * (i - 1) / 2 + (j - i);
        if (P.DinvP) P.DinvP[pk] = t;
        if (P.DinvP32) P.DinvP32[pk] = (float)t;
      }
    }
    // facet geometry from the first neighbour's sorted vertices
    if (threadIdx.x == 0) {
      if (!ok) atomicOr(P.status, 2);
      int64_t e = P.facet_el[2 * g];
      int sl = P.facet_slot[2 * g];
      int c = 0;
      for (int j = 0; j < nv; ++j)
        if (j != sl) {
          int v = P.elem_verts[e * nv + j];
          for (int r = 0; r < 3; ++r) X[c][r] = r < d ? P.coords[(size_t)v * d + r] : 0.0;
          ++c;
        }
      double t1[3], t2[3], n[3];
      for (int r = 0; r < 3; ++r) { t1[r] = X[1][r] - X[0][r]; t2[r] = (d == 3) ? X[2][r] - X[0][r] : 0.0; }
      double area;
      if (d == 2) {
        n[0] = t1[1]; n[1] = -t1[0]; n[2] = 0.0;
        area = sqrt(t1[0] * t1[0] + t1[1] * t1[1]);
      } else {
        n[0] = t1[1] * t2[2] - t1[2] * t2[1];
        n[1] = t1[2] * t2[0] - t1[0] * t2[2];
        n[2] = t1[0] * t2[1] - t1[1] * t2[0];
        area = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      }
      double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int r = 0; r < 3; ++r) geo[r] = n[r] / nn;
      geo[3] = area;
      // tangential coordinates of P_t e_c: solve Gram(t) a = (t_b . e_c)
      if (d == 2) {
        double tt = t1[0] * t1[0] + t1[1] * t1[1];
        for (int cc = 0; cc < 2; ++cc) geo[4 + cc] = t1[cc] / tt;   // a_0(c)
      } else {
        double g11 = t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2];
        double g12 = t1[0] * t2[0] + t1[1] * t2[1] + t1[2] * t2[2];
        double g22 = t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2];
        double det = g11 * g22 - g12 * g12;
        for (int cc = 0; cc < 3; ++cc) {
          double r1 = t1[cc], r2 = t2[cc];
          geo[4 + cc] = (g22 * r1 - g12 * r2) / det;        // a_0(c)
          geo[7 + cc] = (-g12 * r1 + g11 * r2) / det;       // a_1(c)
        }
      }
    }
    __syncthreads();
    const int dd = d * d;
    for (int idx = threadIdx.x; idx < nfb * dd; idx += blockDim.x) {
      int q = idx / dd, vc = idx % dd, v = vc / d, c = vc % d;
      double val;
      if (q < s.nF) {
        val = geo[3] * geo[c] * P.rcn[q * d + v];
      } else if (q >= s.nF + s.nh) {
        // k = 1: the flux of curl(lambda_v e_c) through F w.r.t. n_F, by
        // Stokes the circulation of lambda_v e_c along dF (X_0 -> X_1 -> X_2,
        // positive about n_F): (1/2) e_c . (X_{v+1} - X_{v-1})
        val = 0.5 * (X[(v + 1) % 3][c] - X[(v + 2) % 3][c]);
      } else if (P.facet_out && P.facet_out[g]) {
        val = 0.0;   // pi_0 (Lemma outflow): the outlet's tangential dofs stay zero
      } else {
        int j = q - s.nF, b = j / s.nFkm1, gm = j % s.nFkm1;
        val = P.rct[gm * d + v] * geo[4 + 3 * b + c];
      }
      P.EF[(size_t)g * nfb * dd + idx] = val;
      P.EF32[(size_t)g * nfb * dd + idx] = (float)val;
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// P1 multigrid setup on the vertex lattice.  Stencil entry index of offset
// o in {-1,0,1}^d: sum_a (o_a + 1) 3^a; blocks are d x d (row comp, col comp).
// --------------------------------------------------------------------------
__device__ inline void lat_coords(int64_t v, const int* N, int c[3]) {
  c[0] = (int)(v % N[0]);
  c[1] = (int)((v / N[0]) % N[1]);
  c[2] = (int)(v / ((int64_t)N[0] * N[1]));
}


// A-bar stencil on the finest level: vertex-centric sum over incident elements
// of nu_T int eps(lambda_v e_c) : eps(lambda_w e_e).
// One lattice block per blockIdx.y (all blocks of the finest level).
__global__ void k_p1_assemble(P1Params P) {
  const int d = P.d, nv = d + 1, st = d == 3 ? 27 : 9, dd = d * d;
  const MGBlockDev B = load_block(P.blk + (blockIdx.y));
  int N[3] = {B.n[0] + 1, B.n[1] + 1, B.n[2] + 1};
  for (int64_t lv_ = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; lv_ < B.nvert; lv_ += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = B.voff + lv_;
    double* Av = P.A + (size_t)v * st * dd;
    for (int i = 0; i < st * dd; ++i) Av[i] = 0.0;
    int cv[3];
    lat_coords(lv_, N, cv);
    for (int p = P.vert_elem_off[v]; p < P.vert_elem_off[v + 1]; ++p) {
      int64_t e = P.vert_elem[p];
      // geometry
      double X[4][3], J[3][3], Ji[3][3];
      for (int j = 0; j < nv; ++j) {
        int vv = P.elem_verts[e * nv + j];
        for (int r = 0; r < 3; ++r) X[j][r] = r < d ? P.coords[(size_t)vv * d + r] : 0.0;
      }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = (r < d && c < d) ? X[c + 1][r] - X[0][r] : (r == c ? 1.0 : 0.0);
      double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      double vol = fabs(det) / (d == 2 ? 2.0 : 6.0);
      double gl[4][3];
      for (int r = 0; r < 3; ++r) {
        gl[0][r] = 0.0;
        for (int j = 1; j < nv; ++j) { gl[j][r] = r < d ? Ji[j - 1][r] : 0.0; gl[0][r] -= gl[j][r]; }
      }
      int lv = 0;
      for (int j = 0; j < nv; ++j)
        if (P.elem_verts[e * nv + j] == v) lv = j;
      double w = P.nu[e] * vol;
      for (int j = 0; j < nv; ++j) {
        int cw[3];
        lat_coords(P.elem_verts[e * nv + j] - B.voff, N, cw);
        int o = 0, pw = 1;
        for (int a = 0; a < d; ++a) { o += (cw[a] - cv[a] + 1) * pw; pw *= 3; }
        double gg = 0.0;
        for (int r = 0; r < d; ++r) gg += gl[lv][r] * gl[j][r];
        for (int c = 0; c < d; ++c)
          for (int ee = 0; ee < d; ++ee)
            Av[o * dd + c * d + ee] += w * 0.5 * ((c == ee ? gg : 0.0) + gl[j][c] * gl[lv][ee]);
      }
      // tangential penalty on the element's facets on outlet faces (Lemma
      // outflow): nu_T C k^2 / h int_F (lambda_v e_c)_t . (lambda_w e_e)_t,
      // h = d |T| / |F|
      if (B.ffm)
        for (int f = 0; f < nv; ++f) {
          if (f == lv) continue;
          bool on = false;
          for (int a = 0; a < d && !on; ++a)
            for (int side = 0; side < 2 && !on; ++side) {
              if (!((B.ffm >> (2 * a + side)) & 1)) continue;
              bool all = true;
              for (int j = 0; j < nv; ++j) {
                if (j == f) continue;
                int cj[3];
                lat_coords(P.elem_verts[e * nv + j] - B.voff, N, cj);
                if (cj[a] != (side ? B.n[a] : 0)) all = false;
              }
              on = all;
            }
          if (!on) continue;
          int fv[3], m = 0;
          for (int j = 0; j < nv; ++j)
            if (j != f) fv[m++] = j;
          double t1[3], t2[3], nf[3];
          for (int r = 0; r < 3; ++r) {
            t1[r] = X[fv[1]][r] - X[fv[0]][r];
            t2[r] = d == 3 ? X[fv[2]][r] - X[fv[0]][r] : 0.0;
          }
          double area;
          if (d == 2) {
            nf[0] = t1[1];
            nf[1] = -t1[0];
            nf[2] = 0.0;
          } else {
            nf[0] = t1[1] * t2[2] - t1[2] * t2[1];
            nf[1] = t1[2] * t2[0] - t1[0] * t2[2];
            nf[2] = t1[0] * t2[1] - t1[1] * t2[0];
          }
          const double nn = sqrt(nf[0] * nf[0] + nf[1] * nf[1] + nf[2] * nf[2]);
          area = d == 2 ? nn : 0.5 * nn;
          for (int r = 0; r < 3; ++r) nf[r] /= nn;
          const double h = d * vol / area;
          const double cf = P.nu[e] * P.penalty * P.k * P.k / h;
          for (int j = 0; j < nv; ++j) {
            if (j == f) continue;
            int cw[3];
            lat_coords(P.elem_verts[e * nv + j] - B.voff, N, cw);
            int o = 0, pw = 1;
            for (int a = 0; a < d; ++a) { o += (cw[a] - cv[a] + 1) * pw; pw *= 3; }
            const double mass = area * (j == lv ? 2.0 : 1.0) / (d * (d + 1));
            for (int c = 0; c < d; ++c)
              for (int ee = 0; ee < d; ++ee)
                Av[o * dd + c * d + ee] += cf * mass * ((c == ee ? 1.0 : 0.0) - nf[c] * nf[ee]);
          }
        }
    }
  }
}

// l1 block-Jacobi inverse: D_v = A_vv + diag(sum over free w != v of |A_vw| row sums),
// on the continuing blocks of a level (one block per blockIdx.y).
__global__ void k_mg_l1(MGSetupParams P) {
  const int d = P.d, st = d == 3 ? 27 : 9, dd = d * d;
  const MGBlockDev B = load_block(P.blk + (blockIdx.y));
  int N[3] = {B.n[0] + 1, B.n[1] + 1, B.n[2] + 1};
  for (int64_t lv_ = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; lv_ < B.nvert; lv_ += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = B.voff + lv_;
    int cv[3];
    lat_coords(lv_, N, cv);
    double Dm[3][3] = {};
    if (lat_free(cv, B.n, d, B.ffm)) {
      const double* Av = P.A + (size_t)v * st * dd;
      int center = d == 3 ? 13 : 4;
      for (int c = 0; c < d; ++c)
        for (int e = 0; e < d; ++e) Dm[c][e] = Av[center * dd + c * d + e];
      for (int o = 0; o < st; ++o) {
        if (o == center) continue;
        int cw[3] = {cv[0] + o % 3 - 1, cv[1] + (o / 3) % 3 - 1, cv[2] + (o / 9) - 1};
        if (d == 2) cw[2] = 0;
        if (!lat_free(cw, B.n, d, B.ffm)) continue;
        for (int c = 0; c < d; ++c) {
          double sacc = 0.0;
          for (int e = 0; e < d; ++e) sacc += fabs(Av[o * dd + c * d + e]);
          Dm[c][c] += sacc;
        }
      }
    } else {
      for (int c = 0; c < d; ++c) Dm[c][c] = 1.0;
    }
    double inv[3][3];
    if (d == 2) {
      double det = Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0];
      inv[0][0] = Dm[1][1] / det; inv[0][1] = -Dm[0][1] / det;
      inv[1][0] = -Dm[1][0] / det; inv[1][1] = Dm[0][0] / det;
    } else {
      double det = Dm[0][0] * (Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1]) - Dm[0][1] * (Dm[1][0] * Dm[2][2] - Dm[1][2] * Dm[2][0]) +
                   Dm[0][2] * (Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]);
      inv[0][0] = (Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1]) / det;
      inv[0][1] = (Dm[0][2] * Dm[2][1] - Dm[0][1] * Dm[2][2]) / det;
      inv[0][2] = (Dm[0][1] * Dm[1][2] - Dm[0][2] * Dm[1][1]) / det;
      inv[1][0] = (Dm[1][2] * Dm[2][0] - Dm[1][0] * Dm[2][2]) / det;
      inv[1][1] = (Dm[0][0] * Dm[2][2] - Dm[0][2] * Dm[2][0]) / det;
      inv[1][2] = (Dm[0][2] * Dm[1][0] - Dm[0][0] * Dm[1][2]) / det;
      inv[2][0] = (Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]) / det;
      inv[2][1] = (Dm[0][1] * Dm[2][0] - Dm[0][0] * Dm[2][1]) / det;
      inv[2][2] = (Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0]) / det;
    }
    for (int c = 0; c < d; ++c)
      for (int e = 0; e < d; ++e) {
        P.Dinv[(size_t)v * dd + c * d + e] = inv[c][e];
        P.Dinv32[(size_t)v * dd + c * d + e] = (float)inv[c][e];
      }
  }
}

__device__ inline int coarse_pos(int I, int n) { return (2 * I < n) ? 2 * I : n; }

// interpolation weight P(i, I) along one axis with n fine intervals
__device__ inline double w1d(int i, int I, int n) {
  int c = coarse_pos(I, n);
  if (i == c) return 1.0;
  bool is_coarse = (i % 2 == 0) || (i == n);
  if (!is_coarse && (i - c == 1 || c - i == 1)) return 0.5;
  return 0.0;
}

// Galerkin coarse operator A_c = P^T A P restricted to interior vertices, on
// the continuing blocks of a level (one block per blockIdx.y).  One 32-lane
// group per coarse vertex; lane co forms the coupling to the coarse
// neighbour co:  A_c[I][co] = sum_{i, j} P(i, I) A[i][j] P(j, I + co).
__global__ void __launch_bounds__(256) k_mg_rap(MGSetupParams P) {
  const int d = P.d, st = d == 3 ? 27 : 9, dd = d * d;
  const MGBlockDev B = load_block(P.blk + (blockIdx.y));
  int Nf[3] = {B.n[0] + 1, B.n[1] + 1, B.n[2] + 1};
  int Nc[3] = {B.nc3[0] + 1, B.nc3[1] + 1, B.nc3[2] + 1};
  const int co = threadIdx.x & 31;
  const int64_t gpb = blockDim.x >> 5;
  for (int64_t V = blockIdx.x * gpb + (threadIdx.x >> 5); V < B.nvert_c; V += (int64_t)gridDim.x * gpb) {
    if (co >= st) continue;
    double acc[9];
    for (int c = 0; c < dd; ++c) acc[c] = 0.0;
    int CI[3];
    lat_coords(V, Nc, CI);
    int CJ[3] = {CI[0] + co % 3 - 1, CI[1] + (co / 3) % 3 - 1, CI[2] + co / 9 - 1};
    if (d == 2) CJ[2] = 0;
    if (lat_free(CI, B.nc3, d, B.ffm) && lat_free(CJ, B.nc3, d, B.ffm)) {
      int base[3] = {coarse_pos(CI[0], B.n[0]), coarse_pos(CI[1], B.n[1]), d == 3 ? coarse_pos(CI[2], B.n[2]) : 0};
      for (int fo = 0; fo < st; ++fo) {
        int fi[3] = {base[0] + fo % 3 - 1, base[1] + (fo / 3) % 3 - 1, base[2] + fo / 9 - 1};
        if (d == 2) fi[2] = 0;
        if (!lat_free(fi, B.n, d, B.ffm)) continue;
        double wI = 1.0;
        for (int a = 0; a < d; ++a) wI *= w1d(fi[a], CI[a], B.n[a]);
        if (wI == 0.0) continue;
        const int64_t fiv = B.voff + fi[0] + (int64_t)Nf[0] * (fi[1] + (int64_t)Nf[1] * fi[2]);
        const double* Af = P.A + (size_t)fiv * st * dd;
        for (int so = 0; so < st; ++so) {
          int fj[3] = {fi[0] + so % 3 - 1, fi[1] + (so / 3) % 3 - 1, fi[2] + so / 9 - 1};
          if (d == 2) fj[2] = 0;
          if (!lat_free(fj, B.n, d, B.ffm)) continue;
          double wJ = 1.0;
          for (int a = 0; a < d; ++a) wJ *= w1d(fj[a], CJ[a], B.n[a]);
          if (wJ == 0.0) continue;
          for (int c = 0; c < dd; ++c) acc[c] += wI * wJ * Af[so * dd + c];
        }
      }
    }
    double* Ac = P.Ac + (size_t)(B.cvoff + V) * st * dd + co * dd;
    for (int c = 0; c < dd; ++c) Ac[c] = acc[c];
  }
}

__global__ void k_to_f32(const double* a, float* b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (float)a[i];
}

// Coarsest levels: dense matrix over the free dofs of each coarsest block
// (blocks jb .. of the level, one per blockIdx.y), then its inverse (one
// workgroup per block).  Cd/W of block j start at scratch + 2 (cinv_off_j -
// base).
__global__ void k_coarse_gather(MGSetupParams P, int jb, int64_t base, double* scratch) {
  const int d = P.d, st = d == 3 ? 27 : 9, dd = d * d;
  const MGBlockDev B = load_block(P.blk + (P.ncont + jb + blockIdx.y));
  int N[3] = {B.n[0] + 1, B.n[1] + 1, B.n[2] + 1};
  const int64_t nc = B.nc;
  const int32_t* cmap = P.cmap + B.cmap_off;
  double* Cd = scratch + 2 * (B.cinv_off - base);
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nc * nc; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = idx / nc, j = idx % nc;
    int64_t vi = cmap[i] / d, vj = cmap[j] / d;
    int ci = cmap[i] % d, cj = cmap[j] % d;
    int a[3], b[3];
    lat_coords(vi, N, a);
    lat_coords(vj, N, b);
    double v = 0.0;
    bool near = true;
    int o = 0, pw = 1;
    for (int ax = 0; ax < d; ++ax) {
      int df = b[ax] - a[ax];
      if (df < -1 || df > 1) near = false;
      o += (df + 1) * pw;
      pw *= 3;
    }
    if (near) v = P.A[(size_t)(B.voff + vi) * st * dd + o * dd + ci * d + cj];
    Cd[idx] = v;
  }
}

__global__ void __launch_bounds__(1024) k_coarse_invert(MGSetupParams P, int jb, int64_t base, double* scratch,
                                                         double* Cinv_all, int* status) {
  // Cholesky in place (lower), L^{-1} into W, Cinv = L^{-T} L^{-1}.
  const MGBlockDev B = load_block(P.blk + (P.ncont + jb + blockIdx.x));
  const int64_t n = B.nc;
  double* C = scratch + 2 * (B.cinv_off - base);
  double* W = C + n * n;
  double* Cinv = Cinv_all + B.cinv_off;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int64_t j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double v = C[j * n + j];
      if (!(v > 0.0)) { bad = 1; v = 1.0; }
      C[j * n + j] = sqrt(v);
    }
    __syncthreads();
    double piv = C[j * n + j];
    for (int64_t i = j + 1 + threadIdx.x; i < n; i += blockDim.x) C[i * n + j] /= piv;
    __syncthreads();
    int64_t m = n - j - 1;
    for (int64_t idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      int64_t i = j + 1 + idx / m, c = j + 1 + idx % m;
      if (c <= i) C[i * n + c] -= C[i * n + j] * C[c * n + j];
    }
    __syncthreads();
  }
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    for (int64_t i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      if (i > c)
        for (int64_t p = c; p < i; ++p) t -= C[i * n + p] * W[p * n + c];
      W[i * n + c] = (i < c) ? 0.0 : t / C[i * n + i];
    }
  }
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    int64_t i = idx / n, j = idx % n;
    int64_t p0 = i > j ? i : j;
    double t = 0.0;
    for (int64_t p = p0; p < n; ++p) t += W[p * n + i] * W[p * n + j];
    Cinv[idx] = t;
  }
  if (threadIdx.x == 0 && bad) atomicOr(status, 4);
}

// Load vector (f, phi) with f the degree-m lattice interpolant (caller vertex
// order, mapped to the sorted order through the element's permutation).
__global__ void __launch_bounds__(256) k_load(CondParams C, SolveParams P, const int32_t* __restrict__ elem_perm,
                                              const int32_t* __restrict__ latmap, const double* __restrict__ rRf,
                                              const double* __restrict__ f, double* __restrict__ b,
                                              double* __restrict__ escr) {
  const Sizes s = C.s;
  const int d = s.d, nb = s.nb, nd = s.nd;
  __shared__ ElemGeo g;
  __shared__ double Jf[128][3];
  const int tid = threadIdx.x;
  for (int64_t e = blockIdx.x; e < C.ne; e += gridDim.x) {
    if (tid == 0) element_geometry(C, e, g);
    __syncthreads();
    const int pr = elem_perm[e];
    for (int lc = tid; lc < s.nlat; lc += blockDim.x) {
      int ls = latmap[(size_t)pr * s.nlat + lc];
      for (int r = 0; r < d; ++r) {
        double t = 0.0;
        for (int a = 0; a < d; ++a) t += g.J[a][r] * f[((size_t)e * s.nlat + lc) * d + a];
        Jf[ls][r] = t;
      }
    }
    __syncthreads();
    const double adet = fabs(g.det);
    for (int row = tid; row < nb + nd; row += blockDim.x) {
      int iu = -1;
      double sc = 1.0;
      if (row < nb) { iu = row; sc = adet; }
      else {
        int rr = row - nb, ff = rr / s.nfb, q = rr % s.nfb;
        if (q < s.nF) { iu = nb + ff * s.nF + q; sc = adet / g.det; }
      }
      double acc = 0.0;
      if (iu >= 0)
        for (int l = 0; l < s.nlat; ++l)
          for (int r = 0; r < d; ++r) acc += Jf[l][r] * rRf[((size_t)l * s.nu + iu) * d + r];
      acc *= sc;
      if (row < nb) b[e * nb + row] = acc;
      else escr[e * nd + row - nb] = acc;
    }
    __syncthreads();
  }
}

__global__ void k_check_nu(const double* nu, int64_t n, int* status) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = nu[i];
    if (!(v > 0.0) || !(v < 1e300)) atomicOr(status, 8);
  }
}

// Mean of the pressure: red[0] = sum_T |T| sum_q p_q pmom_q, red[1] = |Omega|,
// then p -= mean * pconst (the coefficients of p = 1).
__global__ void __launch_bounds__(256) k_pmean_reduce(SolveParams P, const double* __restrict__ pmom,
                                                      const double* __restrict__ x, double* red) {
  __shared__ double sh[2][256];
  const Sizes s = P.s;
  const double fd = s.d == 2 ? 2.0 : 6.0;
  double a = 0.0, v = 0.0;
  for (int64_t e = threadIdx.x; e < P.ne; e += 256) {
    double vol = fabs(P.detJ[e]) / fd;
    double t = 0.0;
    for (int q = 0; q < s.np; ++q) t += pmom[q] * x[P.off_p + e * s.np + q];
    a += vol * t;
    v += vol;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) red[0] = sh[0][0] / sh[1][0];
}

__global__ void k_pmean_sub(SolveParams P, const double* __restrict__ pconst, const double* __restrict__ red,
                            double* __restrict__ x) {
  const int np = P.s.np;
  const double m = red[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P.ne * np; i += (int64_t)gridDim.x * blockDim.x)
    x[P.off_p + i] -= m * pconst[i % np];
}

// --------------------------------------------------------------------------
// Stress and vorticity recovery (Sec. 4.2, eq. projection) at reference
// points.  In the orthonormal stress basis psi_a D_m (mass matrix (|T|/nu) I)
// the local problems give, with g = G^T u over the reduced columns,
//     sigma = (nu/|T|) (I - Q^T Q) g,
// and the multiplier omega in W_h = P^{k-1}(T, K) has the coefficients
// -(1/|T|) b(psi_a D_m, u) on the skew D_m and the psi_a of degree < k (these
// columns are exactly the ones the reduced space leaves out).  One workgroup
// per element; the slot scratch holds Q and the small vectors.
// --------------------------------------------------------------------------
constexpr int MAXNS = 56;  // dim P^5 in 3D

__global__ void __launch_bounds__(256) k_stress(StressParams S) {
  const CondParams& P = S.C;
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1, tid = threadIdx.x;
  // omega's coefficients (k >= 2: the skew P^{k-1} multiplier, recovered
  // from the local problem; k = 1: omega is global, its facet fluxes are in x)
  const int nW = s.nw ? 0 : s.nskew * s.nsm1;
  __shared__ ElemGeo g;
  __shared__ double sEm[8][3][3];
  __shared__ double sW[4][8][3];
  __shared__ double sTd[4][2][8];
  __shared__ double sS[48 * 48];
  double* Lm = P.scratch + (size_t)blockIdx.x * P.slot_doubles;  // nlam x nsig
  double* ul = Lm + (size_t)s.nlam * s.nsig;                      // nA
  double* gs = ul + s.nA;                                         // nsig
  double* tq = gs + s.nsig;                                       // nlam
  double* wc = tq + s.nlam;                                       // nskew x nsm1
  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    stress_tables(P, e, g, sEm, sW, sTd);
    const double adet = fabs(g.det), idet = 1.0 / g.det;
    for (int i = tid; i < s.nA; i += blockDim.x) {
      double v = 0.0;
      if (i < s.nb) {
        v = S.x[e * s.nb + i];
      } else {
        const int f = (i - s.nb) / s.nfb, q = (i - s.nb) % s.nfb;
        const int gf = S.elem_ff[e * nv + f];
        if (gf >= 0) v = S.x[S.off_f + (int64_t)gf * s.nfb + q];
        else if (S.xD) v = S.xD[e * s.nd + (i - s.nb)];
      }
      ul[i] = v;
    }
    const bool ok = lambda_q(P, sTd, Lm, sS);  // synchronises: ul visible
    for (int c = tid; c < s.nsig + nW; c += blockDim.x) {
      int m, a;
      if (c < s.nsig) sig_col(s, c, m, a);
      else { m = s.nsym + (c - s.nsig) / s.nsm1; a = (c - s.nsig) % s.nsm1; }
      double t = 0.0;
      for (int i = 0; i < s.nA; ++i) t += g_entry(P, g, sEm, sW, sTd, i, m, a, adet, idet) * ul[i];
      if (c < s.nsig) gs[c] = t;
      else wc[c - s.nsig] = -t / g.vol;
    }
    __syncthreads();
    for (int l = tid; l < s.nlam; l += blockDim.x) {
      double t = 0.0;
      for (int c = 0; c < s.nsig; ++c) t += Lm[(size_t)l * s.nsig + c] * gs[c];
      tq[l] = t;
    }
    __syncthreads();
    const double cf = P.nu[e] / g.vol;
    for (int c = tid; c < s.nsig; c += blockDim.x) {
      double t = gs[c];
      for (int l = 0; l < s.nlam; ++l) t -= Lm[(size_t)l * s.nsig + c] * tq[l];
      gs[c] = cf * t;
    }
    __syncthreads();
    // caller order of the sorted vertices
    int perm[4];
    {
      int r = S.elem_perm[e], dig[4], avail[4];
      for (int i = nv - 1; i >= 0; --i) {
        dig[i] = r % (nv - i);
        r /= (nv - i);
      }
      for (int i = 0; i < nv; ++i) avail[i] = i;
      int na = nv;
      for (int i = 0; i < nv; ++i) {
        perm[i] = avail[dig[i]];
        for (int j = dig[i]; j + 1 < na; ++j) avail[j] = avail[j + 1];
        --na;
      }
    }
    for (int q = tid; q < S.npts; q += blockDim.x) {
      double lam[4], mono[MAXNS], psi[MAXNS];
      for (int j = 0; j < nv; ++j) lam[j] = S.pts[q * nv + perm[j]];
      for (int j = 0; j < s.ns; ++j) {
        double v = 1.0;
        for (int t = 0; t < nv; ++t)
          for (int p = 0; p < (int)S.rpsib[j * nv + t]; ++p) v *= lam[t];
        mono[j] = v;
      }
      for (int a = 0; a < s.ns; ++a) {
        double v = 0.0;
        for (int j = 0; j < s.ns; ++j) v += S.rpsi[(size_t)a * s.ns + j] * mono[j];
        psi[a] = v;
      }
      double sg[3][3] = {}, om[3][3] = {};
      const int ntop = s.ns - s.sklo;
      for (int m = 0; m < s.nsym + s.nskew; ++m) {
        double cs = 0.0, cw = 0.0;
        if (m < s.nsym) {
          for (int a = 0; a < s.ns; ++a) cs += gs[m * s.ns + a] * psi[a];
        } else {
          const int mk = m - s.nsym;
          for (int a = 0; a < ntop; ++a) cs += gs[s.nsym * s.ns + mk * ntop + a] * psi[s.sklo + a];
          for (int a = 0; a < nW / s.nskew; ++a) cw += wc[mk * s.nsm1 + a] * psi[a];
        }
        double D[3][3];
        dm_basis(d, m, D);
        for (int r = 0; r < d; ++r)
          for (int c = 0; c < d; ++c) {
            sg[r][c] += cs * D[r][c];
            om[r][c] += cw * D[r][c];
          }
      }
      if (s.nw) {
        // k = 1: omega_h = sum_f flux_f s_f (x - x_f) / (d |T|) with
        // x - x_f = sum_j lambda_j (x_j - x_f); the output is kappa(omega_h)
        double w[3] = {0.0, 0.0, 0.0};
        for (int f = 0; f < nv; ++f) {
          const double cf = ul[s.nb + f * s.nfb + s.nF + s.nh] * rt_sign(g, f) / (d * g.vol);
          for (int j = 0; j < nv; ++j)
            for (int r = 0; r < 3; ++r) w[r] += cf * lam[j] * (g.X[j][r] - g.X[f][r]);
        }
        om[0][1] = -0.5 * w[2];
        om[0][2] = 0.5 * w[1];
        om[1][0] = 0.5 * w[2];
        om[1][2] = -0.5 * w[0];
        om[2][0] = -0.5 * w[1];
        om[2][1] = 0.5 * w[0];
      }
      const size_t o = ((size_t)e * S.npts + q) * d * d;
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
          S.sig[o + r * d + c] = sg[r][c];
          S.om[o + r * d + c] = om[r][c];
        }
    }
    if (tid == 0 && !ok) atomicOr(P.status, 1);
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// Full-system variant (Theorem aux_pc): overlapping facet blocks of A, the
// bubble rows of the embedding E and W_T = A_T E_T.
// --------------------------------------------------------------------------
// Local rows of entry j of block b in its two neighbours (-1: not there):
// facet dofs first, then the bubbles of the first and of the second neighbour.
__device__ inline void full_entry(const Sizes& s, int nf, int s0, int s1, bool two, int j, int& l0, int& l1) {
  if (j < nf) {
    l0 = s.nb + s0 * s.nfb + j;
    l1 = two ? s.nb + s1 * s.nfb + j : -1;   // outlet facets: one neighbour
  } else if (j < nf + s.nb) {
    l0 = j - nf;
    l1 = -1;
  } else {
    l0 = -1;
    l1 = j - nf - s.nb;
  }
}

// Binv[b] = D_B^{-1}, D_B = A restricted to the dofs of block b (assembled
// from the neighbours' A_T; bubbles of different elements do not couple).
__global__ void __launch_bounds__(256) k_full_blocks(Sizes s, FullDev F, int* status) {
  constexpr int FLD = 64;
  __shared__ double S[FLD * FLD];
  __shared__ double W[FLD * FLD];
  const int nA = s.nA, nbk = F.nbk;
  for (int64_t b = blockIdx.x; b < F.nblk; b += gridDim.x) {
    const int64_t e0 = F.blk_el[2 * b], e1 = F.blk_el[2 * b + 1];
    const int s0 = F.blk_slot[2 * b], s1 = F.blk_slot[2 * b + 1];
    const bool two = e1 >= 0;
    const int nf = F.blk_g[b] >= 0 ? s.nfb : 0;
    const int m = nf + s.nb * (two ? 2 : 1);
    const double* A0 = F.A + (size_t)e0 * nA * nA;
    const double* A1 = two ? F.A + (size_t)e1 * nA * nA : nullptr;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int i = idx / m, j = idx % m;
      int a0, a1, c0, c1;
      full_entry(s, nf, s0, s1, two, i, a0, a1);
      full_entry(s, nf, s0, s1, two, j, c0, c1);
      double v = 0.0;
      if (a0 >= 0 && c0 >= 0) v += A0[(size_t)a0 * nA + c0];
      if (a1 >= 0 && c1 >= 0) v += A1[(size_t)a1 * nA + c1];
      S[i * FLD + j] = v;
    }
    __syncthreads();
    const bool ok = block_cholesky(S, m, FLD);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) W[(idx / m) * FLD + idx % m] = (idx / m == idx % m) ? 1.0 : 0.0;
    __syncthreads();
    block_trsm_lower(S, FLD, W, FLD, m, m);
    for (int idx = threadIdx.x; idx < nbk * nbk; idx += blockDim.x) {
      const int i = idx / nbk, j = idx % nbk;
      double t = 0.0;
      if (i < m && j < m) {
        const int p0 = i > j ? i : j;
        for (int p = p0; p < m; ++p) t += W[p * FLD + i] * W[p * FLD + j];
      }
      F.Binv[(size_t)b * nbk * nbk + idx] = t;
    }
    if (threadIdx.x == 0 && !ok) atomicOr(status, 2);
    __syncthreads();
  }
}

// Bubble rows of E_T: Eo[e][i][vl*d + c] = sum_r (J^{-1})_{r c} Eo_ref[vl][r][i]
// (lambda_v e_c = J (lambda_v J^{-1} e_c) and bubbles map as phi = J phi^).
__global__ void k_full_eo(Sizes s, int64_t ne, FullDev F, const int32_t* __restrict__ elem_verts,
                          const double* __restrict__ coords) {
  const int d = s.d, nv = d + 1, nvd = nv * d;
  const int64_t n = ne * s.nb * nvd;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / (s.nb * nvd);
    const int i = (int)((idx / nvd) % s.nb), m = (int)(idx % nvd), vl = m / d, c = m % d;
    double X[4][3], J[3][3];
    for (int j = 0; j < nv; ++j) {
      const int v = elem_verts[e * nv + j];
      for (int r = 0; r < 3; ++r) X[j][r] = r < d ? coords[(size_t)v * d + r] : 0.0;
    }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) J[r][q] = (r < d && q < d) ? X[q + 1][r] - X[0][r] : (r == q ? 1.0 : 0.0);
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    // column c of J^{-1} (cofactors)
    double Jic[3];
    {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      for (int r = 0; r < 3; ++r) {
        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
        Jic[r] = (J[c1][r1] * J[c2][r2] - J[c1][r2] * J[c2][r1]) / det;
      }
    }
    double t = 0.0;
    for (int r = 0; r < d; ++r) t += Jic[r] * F.Eo_ref[((size_t)vl * d + r) * s.nb + i];
    F.Eo[idx] = t;
  }
}

// W[e][m][row] = sum_j A_T[row][j] E_T[j][m] over the bubble rows (Eo) and the
// facet rows of the free facets (EF).
__global__ void __launch_bounds__(256) k_full_w(Sizes s, int64_t ne, FullDev F, const int32_t* __restrict__ elem_ff,
                                                const double* __restrict__ EF) {
  const int d = s.d, nv = d + 1, nvd = nv * d, nA = s.nA, nfb = s.nfb, dd = d * d;
  for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
    for (int idx = threadIdx.x; idx < nA * nvd; idx += blockDim.x) {
      const int m = idx / nA, row = idx % nA;
      const int vl = m / d, c = m % d;
      const double* Ar = F.A + ((size_t)e * nA + row) * nA;
      double acc = 0.0;
      for (int j = 0; j < s.nb; ++j) acc += Ar[j] * F.Eo[((size_t)e * s.nb + j) * nvd + m];
      for (int f = 0; f < nv; ++f) {
        const int g = elem_ff[e * nv + f];
        if (g < 0 || vl == f) continue;
        const int v = vl < f ? vl : vl - 1;
        const double* E = EF + (size_t)g * nfb * dd + v * d + c;
        for (int q = 0; q < nfb; ++q) acc += Ar[s.nb + f * nfb + q] * E[(size_t)q * dd];
      }
      F.W[((size_t)e * nvd + m) * nA + row] = acc;
    }
  }
}

static int sgrid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65535 * 8));
}

void launch_condense(hipStream_t st, const CondParams& P, int nslots) {
  hipLaunchKernelGGL(k_condense, dim3(nslots), dim3(256), 0, st, P);
}
void launch_full_setup(hipStream_t st, const Sizes& s, int64_t ne, const FullDev& F, const int32_t* elem_verts,
                       const double* coords, const int32_t* elem_ff, const double* EF, int* status) {
  hipLaunchKernelGGL(k_full_eo, dim3(sgrid(ne * s.nb * (s.d + 1) * s.d)), dim3(256), 0, st, s, ne, F, elem_verts, coords);
  hipLaunchKernelGGL(k_full_blocks, dim3((unsigned)std::min<int64_t>(F.nblk, 1 << 20)), dim3(256), 0, st, s, F, status);
  hipLaunchKernelGGL(k_full_w, dim3((unsigned)std::min<int64_t>(ne, 1 << 20)), dim3(256), 0, st, s, ne, F, elem_ff, EF);
}
void launch_stress(hipStream_t st, const StressParams& S, int nslots) {
  hipLaunchKernelGGL(k_stress, dim3(nslots), dim3(256), 0, st, S);
}
void launch_facet_setup(hipStream_t st, const FacetSetupParams& P) {
  hipLaunchKernelGGL(k_facet_setup, dim3((int)std::min<int64_t>(P.nff, 1 << 20)), dim3(256), 0, st, P);
}
static unsigned ygrid(int64_t n, int per, int cap = 4096) {
  int64_t g = (n + per - 1) / per;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}
void launch_p1_assemble(hipStream_t st, const P1Params& P) {
  if (P.nblk == 0) return;
  hipLaunchKernelGGL(k_p1_assemble, dim3(ygrid(P.maxv, 256), P.nblk), dim3(256), 0, st, P);
}
void launch_mg_l1(hipStream_t st, const MGSetupParams& P) {
  if (P.ncont == 0) return;
  hipLaunchKernelGGL(k_mg_l1, dim3(ygrid(P.maxv, 256), P.ncont), dim3(256), 0, st, P);
}
void launch_mg_rap(hipStream_t st, const MGSetupParams& P) {
  if (P.ncont == 0) return;
  hipLaunchKernelGGL(k_mg_rap, dim3(ygrid(P.maxvc, 8), P.ncont), dim3(256), 0, st, P);
}
void launch_coarse(hipStream_t st, const MGSetupParams& P, int jb, int nj, int64_t base, double* scratch,
                   double* Cinv, int* status) {
  if (nj == 0) return;
  hipLaunchKernelGGL(k_coarse_gather, dim3(ygrid(P.maxnc * P.maxnc, 256, 1024), nj), dim3(256), 0, st, P, jb, base,
                     scratch);
  hipLaunchKernelGGL(k_coarse_invert, dim3(nj), dim3(1024), 0, st, P, jb, base, scratch, Cinv, status);
}
void launch_to_f32(hipStream_t st, const double* a, float* b, int64_t n) {
  hipLaunchKernelGGL(k_to_f32, dim3(sgrid(n)), dim3(256), 0, st, a, b, n);
}
void launch_load(hipStream_t st, const CondParams& C, const SolveParams& P, const int32_t* elem_perm,
                 const int32_t* latmap, const double* rRf, const double* f, double* b, double* escr) {
  hipLaunchKernelGGL(k_load, dim3((int)std::min<int64_t>(C.ne, 1 << 20)), dim3(256), 0, st, C, P, elem_perm, latmap,
                     rRf, f, b, escr);
}
void launch_check_nu(hipStream_t st, const double* nu, int64_t n, int* status) {
  hipLaunchKernelGGL(k_check_nu, dim3(sgrid(n)), dim3(256), 0, st, nu, n, status);
}
void launch_pressure_mean(hipStream_t st, const SolveParams& P, const double* pmom, const double* pconst, double* x,
                          double* red) {
  hipLaunchKernelGGL(k_pmean_reduce, dim3(1), dim3(256), 0, st, P, pmom, (const double*)x, red);
  hipLaunchKernelGGL(k_pmean_sub, dim3(sgrid(P.ne * P.s.np)), dim3(256), 0, st, P, pconst, (const double*)red, x);
}

// W_T = A^d_T E_T: the element's A^d times its rows of the embedding E^d
// (facet blocks E_F placed at the element's local vertices).  Layout
// W[e][m][t], m = local vertex * d + component, t = row of A^d_T.
__global__ void __launch_bounds__(256) k_wsetup(FacetSetupParams P, const int32_t* __restrict__ elem_ff, int64_t ne,
                                                double* __restrict__ W, float* __restrict__ W32) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1, nvd = nv * d, nd = s.nd, nfb = s.nfb, dd = d * d;
  // the element's facet blocks E_F (zero for Dirichlet facets); each thread
  // takes one row t of A^d (read once, as column t: consecutive threads read
  // consecutive words) and forms all (d + 1) d entries W[m][t]
  __shared__ double Es[4 * 51 * 9];
  for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
    for (int i = threadIdx.x; i < nv * nfb * dd; i += blockDim.x) {
      const int f = i / (nfb * dd), r = i % (nfb * dd);
      const int g = elem_ff[e * nv + f];
      Es[i] = g >= 0 ? P.EF[(size_t)g * nfb * dd + r] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nd; t += blockDim.x) {
      double acc[12];
#pragma unroll
      for (int m = 0; m < 12; ++m) acc[m] = 0.0;
      for (int f = 0; f < nv; ++f) {
        for (int q = 0; q < nfb; ++q) {
          const size_t ai = ((size_t)e * nd + f * nfb + q) * nd + t;
          const double a = P.Ad ? P.Ad[ai] : (double)P.Adh[ai] + (double)P.Adl[ai];
          const double* Eq = Es + (f * nfb + q) * dd;
#pragma unroll
          for (int m = 0; m < 12; ++m) {
            if (m >= nvd) break;
            const int vl = m / d, c = m % d;
            if (vl == f) continue;
            const int v = vl < f ? vl : vl - 1;
            acc[m] += a * Eq[v * d + c];
          }
        }
      }
      for (int m = 0; m < nvd; ++m) {
        if (W) W[((size_t)e * nvd + m) * nd + t] = acc[m];
        W32[((size_t)e * nvd + m) * nd + t] = (float)acc[m];
      }
    }
    __syncthreads();
  }
}

void launch_wsetup(hipStream_t st, const FacetSetupParams& P, const int32_t* elem_ff, int64_t ne, double* W, float* W32) {
  hipLaunchKernelGGL(k_wsetup, dim3((int)std::min<int64_t>(ne, 1 << 20)), dim3(256), 0, st, P, elem_ff, ne, W, W32);
}

}  // namespace mcs
