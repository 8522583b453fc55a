// Solve-phase kernels: element-by-element application of the condensed
// operator through its bubble factorisation (eq. factorSsigma), the pressure
// coupling B (eq. femSPmat), the pieces of A-hat_ext^{-1} (Sec. 6.1), coloured
// facet block Gauss-Seidel sweeps (Theorem aux_pc_schur, Corollary
// aux_pc_mult), the embedding E^d (eq. defED), the P1 lattice V-cycle, and
// vector reductions for MINRES.
//
// Layout of element operators (element-major, row-major inside an element):
//   Ad  [nd][nd] symmetric;  H [nb][nd];
//   Aoo [nb][nb], Aooinv [nb][nb] symmetric;  Dinv [nfb][nfb] symmetric, and
//   DinvP its upper triangle packed row by row (colour phases).
// Products with a symmetric matrix give each thread one column (= one row),
// or two or four adjacent ones read with one wider load, so consecutive
// threads read consecutive addresses; products with the rows of H give each
// group of lanes one row, lanes over its contiguous columns.
#include <type_traits>

#include "kernels_common.h"
#include "launch.h"

namespace mcs {

template <typename R>
__device__ inline void gather_elem_d(const SolveParams& P, const R* __restrict__ x, int64_t e, R* xd) {
  const Sizes& s = P.s;
  const int nv = s.d + 1;
  for (int t = threadIdx.x; t < s.nd; t += blockDim.x) {
    int f = t / s.nfb, q = t % s.nfb;
    int g = P.elem_ff[e * nv + f];
    xd[t] = g >= 0 ? x[P.off_f + (int64_t)g * s.nfb + q] : (P.xD ? (R)P.xD[e * s.nd + t] : R(0));
  }
}

template <typename R>
__device__ inline R wave_sum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over the 32 lanes of a half-wave group
template <typename R>
__device__ inline R group32_sum(R v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 32);
  return v;
}

template <int L, typename R>
__device__ inline R group_sum(R v) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
  return v;
}

// Row products of a row-major nrow x ncol matrix with an LDS vector: threads
// [t0, t0 + nthr) form groups of L lanes, one group per row (lanes over the
// contiguous columns); epi(i, sum) runs on the group's first lane.  The row
// loop is uniform over the participating waves (t0, nthr multiples of 64).
// A group takes two rows per pass; a lane's entries of both are loaded U at
// a time, all in flight together, then each row is summed in column order
// (so the sums depend neither on U nor on the pairing of rows).
template <int L, typename MA, typename R, typename F>
__device__ inline void rows_times(MA M, size_t m0, int nrow, int ncol, const R* v, int t0, int nthr, F epi,
                                  R* keep = nullptr, int ldk = 0) {
  constexpr int U = sizeof(R) == 8 ? 4 : 8;   // 16 words of two rows in flight per lane
  const int t = threadIdx.x - t0;
  const int g = t / L, l = t % L, ng = nthr / L;
  for (int i0 = 0; i0 < nrow; i0 += 2 * ng) {
    const int ia = i0 + g, ib = i0 + ng + g;
    const bool va = ia < nrow, vb = ib < nrow;
    const size_t ma0 = m0 + (size_t)(va ? ia : 0) * ncol, mb0 = m0 + (size_t)(vb ? ib : 0) * ncol;
    R acca = R(0), accb = R(0);
    for (int jb = l; jb < ncol; jb += U * L) {
      R ma[U], mb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = jb + u * L;
        ma[u] = va && j < ncol ? M(ma0 + j) : R(0);
        mb[u] = vb && j < ncol ? M(mb0 + j) : R(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = jb + u * L;
        if (j < ncol) {
          // the matrix entries are also kept in LDS (row stride ldk) for a later product
          if (va) {
            if (keep) keep[ia * ldk + j] = ma[u];
            acca += ma[u] * v[j];
          }
          if (vb) {
            if (keep) keep[ib * ldk + j] = mb[u];
            accb += mb[u] * v[j];
          }
        }
      }
    }
    acca = group_sum<L>(acca);
    accb = group_sum<L>(accb);
    if (l == 0 && va) epi(ia, acca);
    if (l == 0 && vb) epi(ib, accb);
  }
}

// sum_q T[q st] v[q] over q < n, in order of q; the table entries are loaded
// 8 at a time, all in flight together.
template <typename V>
__device__ inline double dot_strided8(const double* __restrict__ T, size_t st, const V* v, int n) {
  double b = 0.0;
  for (int q0 = 0; q0 < n; q0 += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = q0 + u < n ? T[(size_t)(q0 + u) * st] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q0 + u < n) b += t[u] * (double)v[q0 + u];
  }
  return b;
}
// sum_q Bp^[q][iu] x_p[q] over q < n_p
template <typename R>
__device__ inline double bp_column(const double* __restrict__ T, int nu, int iu, const R* xp, int np) {
  return dot_strided8(T + iu, (size_t)nu, xp, np);
}
// The rows q = wave + 4 r (r >= 0, q < n_p) of sum_iu Bp^[q][iu] us[iu] for
// the calling wave, in order of iu for each row; the table entries of two
// rows (three per lane and row: n_u <= 192) are loaded together.  out(q, sum)
// runs on lane 0.
template <typename F>
__device__ inline void bu_rows(const double* __restrict__ T, int nu, int np, const double* us, int wave, int lane,
                               F out) {
  constexpr int QB = 2;
  for (int q0 = wave; q0 < np; q0 += 4 * QB) {
    double t[QB][3];
#pragma unroll
    for (int r = 0; r < QB; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int q = q0 + 4 * r, iu = lane + 64 * c;
        t[r][c] = q < np && iu < nu ? T[(size_t)q * nu + iu] : 0.0;
      }
#pragma unroll
    for (int r = 0; r < QB; ++r) {
      const int q = q0 + 4 * r;   // uniform over the wave
      if (q < np) {
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (lane + 64 * c < nu) a += t[r][c] * us[lane + 64 * c];
        a = wave_sum(a);
        if (lane == 0) out(q, a);
      }
    }
  }
}

// Per-workgroup table of the velocity rows of an element (reordered local
// order): original BDM index (or -1 for tangential rows) and the kind of
// scale in phi = s J phi^ (0: bubble, s = 1; 1: facet function, s = 1/det J).
__device__ inline void build_rowmap(const Sizes& s, int* rmap) {
  for (int row = threadIdx.x; row < s.nb + s.nd; row += blockDim.x) {
    int iu = -1;
    if (row < s.nb) iu = row;
    else {
      int r = row - s.nb, f = r / s.nfb, qq = r % s.nfb;
      if (qq < s.nF) iu = s.nb + f * s.nF + qq;
    }
    rmap[row] = iu;
  }
}

// flags: 1 = velocity block A (factorised), 2 = + B^T p, 4 = p <- B u, 8 = A^d only,
// 16 = write zero pressure rows when B u is not requested.
// Phase 1: the first ceil(n_d / (64 CP)) waves form A^d x_d (CP rows per
// thread, A^d symmetric so its columns are contiguous; CP = 2 loads two
// adjacent words at once and passes the second row through LDS) while the
// remaining waves form z_o = x_o + H x_d (16-lane groups per row of H);
// phase 2: w_o = A_oo z_o; phase 3: H^T w_o (one column per thread) and the
// pressure coupling.  Every row is summed in the same order for CP = 1 and 2.
// CP = 4 (FP32; n_d / 4 <= 64 rows of quads) splits the columns of A^d over
// two waves (j < ceil(n_d / 2) and the rest), their sums added in phase 3:
// two shorter load chains in place of one.
// B_T[q][row] = -s |det J| Bp^[q][iu(row)] (s = 1 bubble, 1/det J facet row).
template <typename R, typename MA, int FL, int CP>
__global__ void __launch_bounds__(256) k_elem_apply(SolveParams P, MA MAd, MA MH, MA MAoo, const R* __restrict__ x,
                                                    R* __restrict__ y, R* __restrict__ escr, int flags, int ldh) {
  if constexpr (FL >= 0) flags = FL;   // specialised instantiations fold the flag tests
  // ldh > 0 (instantiations with CP > 1): H is read once; the rows read for
  // z_o = x_o + H x_d are kept in LDS (row stride ldh) for H^T w_o
  extern __shared__ __align__(16) unsigned char ea_lds[];
  R* sH = (CP > 1 && ldh > 0) ? reinterpret_cast<R*>(ea_lds) : nullptr;
  const Sizes s = P.s;
  const int nb = s.nb, nd = s.nd, np = s.np, nu = s.nu;
  __shared__ R xd[MAXND], xo[MAXNB], zo[MAXNB], wo[MAXNB];
  __shared__ R xp[MAXNP];
  __shared__ int rmap[MAXNB + MAXND];
  __shared__ double us[MAXNB + MAXND];   // Piola-scaled velocity for B u, by BDM index
  constexpr int KS = CP == 4 ? 2 : 1;     // column slices of the A^d product
  __shared__ R adx[CP > 1 ? KS * MAXND : 1];   // A^d x_d (CP > 1), per slice
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool doA = flags & 1, doBT = flags & 2, doBu = flags & 4, onlyAd = flags & 8;
  const bool doH = doA && !onlyAd;
  build_rowmap(s, rmap);
  const int nq = nd / CP;
  constexpr bool split = KS == 2;   // n_d <= MAXND = 256: n_q <= 64 rows of quads
  const int tA = split ? 128 : ((nq + 63) >> 6) << 6;     // threads of the A^d product
  const bool overlap = tA < 256;
  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    if (elem_off(P, e)) continue;
    const double det = P.detJ[e];
    const double sb = -fabs(det), sf = det > 0 ? -1.0 : 1.0;
    if (doA || doBu) {   // B^T p alone needs only the pressure values
      gather_elem_d(P, x, e, xd);
      if (tid < nb) xo[tid] = x[e * nb + tid];
    }
    if (tid < np) xp[tid] = x[P.off_p + e * np + tid];
    __syncthreads();
    const size_t h0 = (size_t)e * nb * nd;
    R acc = R(0);
    if constexpr (CP > 1) {
      // batches of U columns: a batch's loads are issued together, then
      // summed in order (columns past the range load its last one and add it
      // times 0; the sums run over j in order)
      typedef R rcv __attribute__((ext_vector_type(CP)));
      if constexpr (split) {
        // wave sl takes the columns [jlo, jhi) of the rows [CP qq, CP qq + CP)
        constexpr int U = 8;   // registers: still 4 waves per SIMD
        const int sl = tid >> 6, qq = tid & 63;
        const int half = (nd + 1) / 2, jlo = sl * half, jhi = min(nd, jlo + half);
        if (tid < tA && qq < nq && doA) {
          const R* a0 = MAd.p + (size_t)e * nd * nd + CP * qq;
          R ac[CP];
#pragma unroll
          for (int c = 0; c < CP; ++c) ac[c] = R(0);
          for (int jb = jlo; jb < jhi; jb += U) {
            rcv b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) b[u] = *reinterpret_cast<const rcv*>(a0 + (size_t)min(jb + u, jhi - 1) * nd);
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const R xj = xd[min(jb + u, jhi - 1)] * R(jb + u < jhi ? 1 : 0);
#pragma unroll
              for (int c = 0; c < CP; ++c) ac[c] += b[u][c] * xj;
            }
          }
#pragma unroll
          for (int c = 0; c < CP; ++c) adx[sl * MAXND + CP * qq + c] = ac[c];
        }
      } else if (tid < nd / CP) {
        if (doA) {
          constexpr int U = 12;
          const R* a0 = MAd.p + (size_t)e * nd * nd + CP * tid;
          R ac[CP];
#pragma unroll
          for (int c = 0; c < CP; ++c) ac[c] = R(0);
          for (int jb = 0; jb < nd; jb += U) {
            rcv b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) b[u] = *reinterpret_cast<const rcv*>(a0 + (size_t)min(jb + u, nd - 1) * nd);
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const R xj = xd[min(jb + u, nd - 1)] * R(jb + u < nd ? 1 : 0);
#pragma unroll
              for (int c = 0; c < CP; ++c) ac[c] += b[u][c] * xj;
            }
          }
#pragma unroll
          for (int c = 0; c < CP; ++c) adx[CP * tid + c] = ac[c];
        }
      }
    }
    if (CP == 1 && tid < nd) {
      if (doA) {
        const size_t a0 = (size_t)e * nd * nd + tid;
#pragma unroll 8
        for (int j = 0; j < nd; ++j) acc += MAd(a0 + (size_t)j * nd) * xd[j];
      }
    } else if (doH && overlap && tid >= tA) {
      // one wave left for H (n_d > 128): 4-lane groups, 16 rows at a time
      if (256 - tA >= 128)
        rows_times<16>(MH, h0, nb, nd, xd, tA, 256 - tA, [&](int i, R v) { zo[i] = xo[i] + v; }, sH, ldh);
      else
        rows_times<4>(MH, h0, nb, nd, xd, tA, 256 - tA, [&](int i, R v) { zo[i] = xo[i] + v; }, sH, ldh);
    }
    if (doBu) {
      for (int row = tid; row < nb + nd; row += blockDim.x) {
        int iu = rmap[row];
        if (iu >= 0) us[iu] = (row < nb ? sb * (double)xo[row] : sf * (double)xd[row - nb]);
      }
    }
    if (doH && !overlap) {
      __syncthreads();
      rows_times<16>(MH, h0, nb, nd, xd, 0, 256, [&](int i, R v) { zo[i] = xo[i] + v; }, sH, ldh);
    }
    __syncthreads();
    if (doH) {
      rows_times<8>(MAoo, (size_t)e * nb * nb, nb, nb, zo, 0, 256, [&](int i, R v) { wo[i] = v; });
      __syncthreads();
    }
    if (tid < nd) {
      if constexpr (CP > 1) acc = doA ? (split ? adx[tid] + adx[MAXND + tid] : adx[tid]) : R(0);
      if (doH) {
        if (sH) {
#pragma unroll 4
          for (int i = 0; i < nb; ++i) acc += sH[i * ldh + tid] * wo[i];
        } else {
#pragma unroll 4
          for (int i = 0; i < nb; ++i) acc += MH(h0 + tid + (size_t)i * nd) * wo[i];
        }
      }
      if (doBT) {
        const int iu = rmap[nb + tid];
        if (iu >= 0) {
          const double b = bp_column(P.rBp, nu, iu, xp, np);
          acc += (R)(sf * b);
        }
      }
      escr[e * nd + tid] = acc;
    }
    if (!onlyAd && tid < nb) {
      R a = doH ? wo[tid] : R(0);
      if (doBT) {
        const double b = bp_column(P.rBp, nu, tid, xp, np);
        a += (R)(sb * b);
      }
      y[e * nb + tid] = a;
    }
    if (doBu) {
      bu_rows(P.rBp, nu, np, us, wave, lane, [&](int q, double a) { y[P.off_p + e * np + q] = (R)a; });
    } else if (!onlyAd && tid < np && (flags & 16)) {
      y[P.off_p + e * np + tid] = R(0);
    }
    __syncthreads();
  }
}

// y_F = base_F + sign * (escr[T1][F] + escr[T2][F]) for every free facet dof.
template <typename R>
__global__ void k_facet_sum(SolveParams P, const R* __restrict__ escr, const R* __restrict__ base, R sign,
                            R* __restrict__ y) {
  const Sizes s = P.s;
  const int64_t n = P.nff * s.nfb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t g = idx / s.nfb;
    if (facet_off(P, g)) continue;
    int q = (int)(idx % s.nfb);
    int64_t e1 = P.facet_el[2 * g], e2 = P.facet_el[2 * g + 1];
    int s1 = P.facet_slot[2 * g], s2 = P.facet_slot[2 * g + 1];
    R v = escr[e1 * s.nd + s1 * s.nfb + q];
    if (e2 >= 0) v += escr[e2 * s.nd + s2 * s.nfb + q];   // outlet facets have one neighbour
    R b = base ? base[P.off_f + idx] : R(0);
    y[P.off_f + idx] = b + sign * v;
  }
}

// A-hat_ext^{-1}, first part: escr_T = H_T^T r_o,T (threads [0, n_d), one
// column of H_T each); t_o = Aoo^{-1} r_o (the following n_o threads, or the
// first ones when n_d + n_o exceeds the block).  NR > 0 (n_o <= NR and
// n_d + n_o <= 256): every thread loads its n_o matrix entries at once, right
// after r_o, before the barrier (loads past n_o repeat entry n_o - 1 and are
// not used).
template <typename R, int NR>
__global__ void __launch_bounds__(256) k_ext_pre(SolveParams P, OpPtrs<R> O, const R* __restrict__ r,
                                                 R* __restrict__ to, R* __restrict__ escr) {
  const Sizes s = P.s;
  const int nb = s.nb, nd = s.nd;
  __shared__ R ro[MAXNB];
  const int tid = threadIdx.x;
  const int ob = (nd + nb <= 256) ? nd : 0;
  const bool hcol = tid < nd, arow = tid >= ob && tid < ob + nb;
  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    if (elem_off(P, e)) continue;
    if constexpr (NR > 0) {
      R rv = R(0);
      if (tid < nb) rv = r[e * nb + tid];
      // column tid of H_T (threads < n_d) or row tid - ob of Aoo^{-1}
      R a[NR];
      if (hcol || arow) {
        const R* m = hcol ? O.H + (size_t)e * nb * nd + tid : O.Aooinv + (size_t)e * nb * nb + (tid - ob);
        const size_t st = hcol ? (size_t)nd : (size_t)nb;
#pragma unroll
        for (int q = 0; q < NR; ++q) a[q] = m[(size_t)(q < nb ? q : nb - 1) * st];
      }
      if (tid < nb) ro[tid] = rv;
      __syncthreads();
      if (hcol || arow) {
        R acc = R(0);
#pragma unroll
        for (int q = 0; q < NR; ++q)
          if (q < nb) acc += a[q] * ro[q];
        if (hcol) escr[e * nd + tid] = acc;
        else to[e * nb + tid - ob] = acc;
      }
    } else {
      if (tid < nb) ro[tid] = r[e * nb + tid];
      __syncthreads();
      // column tid of H_T and row tid - ob of Aoo^{-1} (a thread may own
      // both when n_d + n_o > 256): 16 entries loaded at a time (in flight
      // together), then summed in order
      auto colsum = [&](const R* m, size_t st) {
        R acc = R(0);
        for (int q0 = 0; q0 < nb; q0 += 16) {
          R a[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) a[u] = m[(size_t)min(q0 + u, nb - 1) * st];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (q0 + u < nb) acc += a[u] * ro[q0 + u];
        }
        return acc;
      };
      if (hcol) escr[e * nd + tid] = colsum(O.H + (size_t)e * nb * nd + tid, (size_t)nd);
      if (arow) to[e * nb + tid - ob] = colsum(O.Aooinv + (size_t)e * nb * nb + (tid - ob), (size_t)nb);
    }
    __syncthreads();
  }
}

// A-hat_ext^{-1}, last part: y_o = t_o - H_T t_d,T (8-lane groups per row of H_T).
// NC > 0 (n_d <= 8 NC, n_o <= 32 RPG): the 32 groups hold the entries of their
// RPG rows (g, g + 32, ...) in registers, loaded after the facet ids and before
// the facet values.
template <typename R, int NC, int RPG>
__global__ void __launch_bounds__(256) k_ext_post(SolveParams P, OpPtrs<R> O, const R* __restrict__ t,
                                                  const R* __restrict__ to, R* __restrict__ y) {
  const Sizes s = P.s;
  const int nb = s.nb, nd = s.nd;
  __shared__ R td[MAXND];
  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    if (elem_off(P, e)) continue;
    if constexpr (NC > 0) {
      const int g = threadIdx.x >> 3, l = threadIdx.x & 7;
      R a[RPG][NC];
#pragma unroll
      for (int q = 0; q < RPG; ++q) {
        const int row = g + 32 * q < nb ? g + 32 * q : nb - 1;
        const R* h = O.H + (size_t)e * nb * nd + (size_t)row * nd;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
          const int j = l + 8 * m;
          a[q][m] = h[j < nd ? j : nd - 1];
        }
      }
      gather_elem_d(P, t, e, td);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RPG; ++q) {
        R acc = R(0);
#pragma unroll
        for (int m = 0; m < NC; ++m) {
          const int j = l + 8 * m;
          if (j < nd) acc += a[q][m] * td[j];
        }
        acc = group_sum<8>(acc);
        const int row = g + 32 * q;
        if (l == 0 && row < nb) y[e * nb + row] = to[e * nb + row] - acc;
      }
    } else {
      gather_elem_d(P, t, e, td);
      __syncthreads();
      rows_times<8>(MatP<R>{O.H}, (size_t)e * nb * nd, nb, nd, td, 0, 256,
                    [&](int i, R v) { y[e * nb + i] = to[e * nb + i] - v; });
    }
    __syncthreads();
  }
}

// One colour phase of block Gauss-Seidel on A^d with maintained element
// products y_T = A^d_T x_T (race free: facets of one colour share no element):
//   r_F = s_F - y_T1[F] - y_T2[F];  delta = D_F^{-1} r_F;  x_F += delta;
//   y_Ti += A^d_Ti[:, F] delta   (columns of F = rows of F, A^d symmetric).
// A workgroup holds FPW facet teams of T1 = round_up(2 n_d, 64) threads; in a
// team, threads [0, n_d) own the rows of the first neighbour and [n_d, 2 n_d)
// those of the second.  Per facet one 16-byte record names both neighbours
// (loaded one facet ahead); then every load of the facet is issued at once:
// D_F^{-1} (its packed upper triangle of NP words, at most NDV per thread as
// T1 >= 2 n_d >= 6 n_fb, copied to LDS as it is) and the facet's values
// first, the A^d rows last, so that the residual and
// D_F^{-1} r_F are formed while the A^d rows are still in flight.  The loads
// are unconditional, at clamped addresses inside the arrays (lanes without a
// row, teams past the colour's end, the missing neighbour of an outlet facet),
// so that the code stays straight and only the stores are predicated.  The
// LDS buffers alternate between consecutive facets: two barriers per facet.
// Workgroups loop over the colour's facets in steps of the grid, so the launch
// shape (FPW, grid) changes only which team handles a facet, never the
// arithmetic.
template <typename R, int NFB, int FPW, bool OUT>
__global__ void __launch_bounds__(512) k_smooth_y(SolveParams P, OpPtrs<R> O, int32_t c0, int32_t c1,
                                                  R* __restrict__ x, const R* __restrict__ srhs, R* __restrict__ y,
                                                  int T1) {
  constexpr int NP = NFB * (NFB + 1) / 2;
  constexpr int NDV = (NP + 6 * NFB - 1) / (6 * NFB);
  const int nd = P.s.nd;
  __shared__ R rr[2][FPW][NFB + 1];
  __shared__ R dl[2][FPW][NFB];
  // the last entry of rr and dsh takes the writes of lanes without an entry
  __shared__ R dsh[2][FPW][NP + 1];
  const int h = threadIdx.x / T1;
  const int tid = threadIdx.x - h * T1;
  const int side = tid >= nd ? 1 : 0;
  const bool is_row = tid < 2 * nd;
  const int t = is_row ? tid - side * nd : nd - 1;
  const int tq = tid < NFB ? tid : NFB - 1;
  int buf = 0;
  const int64_t step = (int64_t)gridDim.x * FPW;
  auto record = [&](int64_t ci) {
    return *reinterpret_cast<const int4*>(P.colour_desc + 4 * (ci < c1 ? ci : (int64_t)c1 - 1));
  };
  // the record of a team's next facet is loaded one facet ahead
  int4 next = record(c0 + (int64_t)blockIdx.x * FPW + h);
  for (int64_t base = c0 + (int64_t)blockIdx.x * FPW; base < c1; base += step, buf ^= 1) {
    const int64_t ci = base + h;
    bool work = ci < c1;
    const int4 dsc = next;
    next = record(ci + step);
    const int64_t g = dsc.x;
    const int64_t e1 = dsc.y;
    const int s1 = dsc.w & 0xFF;
    // OUT: an outlet facet has no second neighbour (-1); its second-side rows
    // read the first neighbour's and store nothing
    const bool has2 = !OUT || dsc.z >= 0;
    const int64_t e2 = has2 ? (int64_t)dsc.z : e1;
    const int s2 = has2 ? (dsc.w >> 8) & 0xFF : s1;
    if (P.active && work && facet_off(P, g)) work = false;
    if (work && P.work_count && tid == 0) atomicAdd(P.work_count + (blockIdx.x & 255) * 16, 1ull);
    const int64_t e = side ? e2 : e1;
    const int sl = side ? s2 : s1;
    R dv[NDV];
    const R* Di = O.DinvP + (size_t)g * NP;
#pragma unroll
    for (int u = 0; u < NDV; ++u) {
      const int i = tid + u * T1;
      dv[u] = Di[i < NP ? i : NP - 1];
    }
    const int64_t fo = P.off_f + g * NFB + tq;
    const R xo = x[fo];
    const R sv = srhs[fo];
    const R y1 = y[e1 * nd + s1 * NFB + tq];
    const R y2 = y[e2 * nd + s2 * NFB + tq];
    R yv = y[e * nd + t];
    R a[NFB];
    const R* Ab = O.Ad + (size_t)e * nd * nd + (size_t)sl * NFB * nd + t;
#pragma unroll
    for (int q = 0; q < NFB; ++q) a[q] = Ab[(size_t)q * nd];
#pragma unroll
    for (int u = 0; u < NDV; ++u) {
      const int i = tid + u * T1;
      dsh[buf][h][i < NP ? i : NP] = dv[u];
    }
    rr[buf][h][tid < NFB ? tid : NFB] = has2 ? sv - y1 - y2 : sv - y1;
    __syncthreads();
    if (tid < NFB) {
      // row tid of D_F^{-1}: (j, tid) from row j's triangle for j < tid, else (tid, j)
      const int rb = tid * NFB - tid * (tid - 1) / 2 - tid;
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < NFB; ++j) {
        const int pk = j < tid ? j * NFB - j * (j - 1) / 2 - j + tid : rb + j;
        acc += dsh[buf][h][pk] * rr[buf][h][j];
      }
      dl[buf][h][tid] = acc;
      if (work) x[fo] = xo + acc;
    }
    __syncthreads();
    if (work && is_row && (side == 0 || has2)) {
#pragma unroll
      for (int q = 0; q < NFB; ++q) yv += a[q] * dl[buf][h][q];
      y[e * nd + t] = yv;
    }
    // no third barrier: the next facet works in the other buffers, and this
    // one is written again only after the next facet's first barrier, which
    // every wave reaches after its last read here
  }
}

// The colour phase of k_smooth_y in 3D with two columns of the facet's row
// block per thread: every A^d load moves two words (16 bytes in FP64), a team
// is round_up(n_d, 64) threads (half the waves), and each column is updated in
// the same order as in k_smooth_y, so the two kernels give identical results.
template <typename R, int NFB, bool OUT>
__global__ void __launch_bounds__(256) k_smooth_y2(SolveParams P, OpPtrs<R> O, int32_t c0, int32_t c1,
                                                   R* __restrict__ x, const R* __restrict__ srhs,
                                                   R* __restrict__ y) {
  typedef R dbl2v __attribute__((ext_vector_type(2)));
  constexpr int NP = NFB * (NFB + 1) / 2;
  constexpr int ND = 4 * NFB, NH = ND / 2;     // columns per side, pairs per side
  constexpr int T1 = ((2 * NH + 63) / 64) * 64;
  constexpr int NDV = (NP + T1 - 1) / T1;
  __shared__ R rr[2][NFB + 1];
  __shared__ R dl[2][NFB];
  __shared__ R dsh[2][NP + 1];
  const int tid = threadIdx.x;
  const int side = tid >= NH ? 1 : 0;
  const bool is_row = tid < 2 * NH;
  const int t = is_row ? 2 * (tid - side * NH) : ND - 2;   // first of the thread's two columns
  const int tq = tid < NFB ? tid : NFB - 1;
  int buf = 0;
  const int64_t step = gridDim.x;
  auto record = [&](int64_t ci) {
    return *reinterpret_cast<const int4*>(P.colour_desc + 4 * (ci < c1 ? ci : (int64_t)c1 - 1));
  };
  int4 next = record(c0 + (int64_t)blockIdx.x);
  for (int64_t ci = c0 + (int64_t)blockIdx.x; ci < c1; ci += step, buf ^= 1) {
    bool work = true;
    const int4 dsc = next;
    next = record(ci + step);
    const int64_t g = dsc.x;
    const int64_t e1 = dsc.y;
    const int s1 = dsc.w & 0xFF;
    const bool has2 = !OUT || dsc.z >= 0;
    const int64_t e2 = has2 ? (int64_t)dsc.z : e1;
    const int s2 = has2 ? (dsc.w >> 8) & 0xFF : s1;
    if (P.active && facet_off(P, g)) work = false;
    if (work && P.work_count && tid == 0) atomicAdd(P.work_count + (blockIdx.x & 255) * 16, 1ull);
    const int64_t e = side ? e2 : e1;
    const int sl = side ? s2 : s1;
    R dv[NDV];
    const R* Di = O.DinvP + (size_t)g * NP;
#pragma unroll
    for (int u = 0; u < NDV; ++u) {
      const int i = tid + u * T1;
      dv[u] = Di[i < NP ? i : NP - 1];
    }
    const int64_t fo = P.off_f + g * NFB + tq;
    const R xo = x[fo];
    const R sv = srhs[fo];
    const R y1 = y[e1 * ND + s1 * NFB + tq];
    const R y2 = y[e2 * ND + s2 * NFB + tq];
    dbl2v yv = *reinterpret_cast<const dbl2v*>(y + e * ND + t);
    dbl2v a[NFB];
    const R* Ab = O.Ad + (size_t)e * ND * ND + (size_t)sl * NFB * ND + t;
#pragma unroll
    for (int q = 0; q < NFB; ++q) a[q] = *reinterpret_cast<const dbl2v*>(Ab + (size_t)q * ND);
#pragma unroll
    for (int u = 0; u < NDV; ++u) {
      const int i = tid + u * T1;
      dsh[buf][i < NP ? i : NP] = dv[u];
    }
    rr[buf][tid < NFB ? tid : NFB] = has2 ? sv - y1 - y2 : sv - y1;
    __syncthreads();
    if (tid < NFB) {
      const int rb = tid * NFB - tid * (tid - 1) / 2 - tid;
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < NFB; ++j) {
        const int pk = j < tid ? j * NFB - j * (j - 1) / 2 - j + tid : rb + j;
        acc += dsh[buf][pk] * rr[buf][j];
      }
      dl[buf][tid] = acc;
      if (work) x[fo] = xo + acc;
    }
    __syncthreads();
    if (work && is_row && (side == 0 || has2)) {
#pragma unroll
      for (int q = 0; q < NFB; ++q) {
        yv.x += a[q].x * dl[buf][q];
        yv.y += a[q].y * dl[buf][q];
      }
      *reinterpret_cast<dbl2v*>(y + e * ND + t) = yv;
    }
  }
}

// The last colour phase of a Gauss-Seidel application whose element products
// are not used afterwards: x_F += D_F^{-1} (s_F - y_T1,F - y_T2,F) for the
// facets of the colour, without reading the facets' rows of A^d or updating y.
// One thread per row of a facet block; the block's residual and the packed
// D_F^{-1} are summed in the order of the colour phase kernels, so x is
// bitwise the x they give.
template <typename R, int NFB, bool OUT>
__global__ void __launch_bounds__(256) k_smooth_last(SolveParams P, OpPtrs<R> O, int32_t c0, int32_t c1,
                                                     R* __restrict__ x, const R* __restrict__ srhs,
                                                     const R* __restrict__ y) {
  constexpr int NP = NFB * (NFB + 1) / 2;
  const int nd = P.s.nd;
  const int64_t n = (int64_t)(c1 - c0) * NFB;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c0 + idx / NFB;
    const int i = (int)(idx % NFB);
    const int4 dsc = *reinterpret_cast<const int4*>(P.colour_desc + 4 * ci);
    const int64_t g = dsc.x, e1 = dsc.y;
    const int s1 = dsc.w & 0xFF;
    const bool has2 = !OUT || dsc.z >= 0;
    const int64_t e2 = has2 ? (int64_t)dsc.z : e1;
    const int s2 = has2 ? (dsc.w >> 8) & 0xFF : s1;
    if (P.active && facet_off(P, g)) continue;
    const R* Di = O.DinvP + (size_t)g * NP;
    const int64_t f0 = P.off_f + g * NFB;
    const int rb = i * NFB - i * (i - 1) / 2 - i;
    R acc = R(0);
#pragma unroll
    for (int j = 0; j < NFB; ++j) {
      const R sv = srhs[f0 + j];
      const R y1 = y[e1 * nd + s1 * NFB + j];
      const R y2 = y[e2 * nd + s2 * NFB + j];
      const R r = has2 ? sv - y1 - y2 : sv - y1;
      const int pk = j < i ? j * NFB - j * (j - 1) / 2 - j + i : rb + j;
      acc += Di[pk] * r;
    }
    x[f0 + i] = x[f0 + i] + acc;
  }
}

// z_F = D_F^{-1} r_F for every free facet block: the facet block Jacobi of the
// additive variant (Theorem aux_pc_schur); one thread per row of a block.
template <typename R>
__global__ void k_block_jacobi(SolveParams P, OpPtrs<R> O, const R* __restrict__ r, R* __restrict__ z) {
  const int nfb = P.s.nfb;
  const int64_t n = P.nff * nfb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = idx / nfb;
    if (facet_off(P, g)) continue;
    const int i = (int)(idx % nfb);
    const R* Di = O.Dinv + (size_t)g * nfb * nfb + i;
    const R* rf = r + P.off_f + g * nfb;
    R acc = R(0);
    for (int j = 0; j < nfb; ++j) acc += Di[(size_t)j * nfb] * rf[j];
    z[P.off_f + idx] = acc;
  }
}

// y_T += W_T c_T with W_T = A^d_T E_T (E_T: the element's rows of E^d) and
// c_T the P1 coarse correction at the element's vertices (lattice vector; the
// Dirichlet vertices carry no value and are skipped, their lattice entries are
// never written): keeps y_T = A^d_T x_T after x += E^d c.
template <typename R, int D>
__global__ void k_elem_ycorr(SolveParams P, const R* __restrict__ W, const int32_t* __restrict__ elem_verts,
                             const int32_t* __restrict__ vfree_of_lat, const R* __restrict__ x0, R* __restrict__ y) {
  const int d = D > 0 ? D : P.s.d, nv = d + 1, nvd = nv * d, nd = P.s.nd;
  const int64_t n = P.ne * nd;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / nd;
    if (elem_off(P, e)) continue;
    const int t = (int)(idx % nd);
    const R* We = W + (size_t)e * nvd * nd + t;
    R acc = R(0);
    if constexpr (D > 0) {
      // the (d+1) d entries of the row, the vertex ids, their free flags and
      // values: each group of loads issued together (three round trips in
      // place of one chain per vertex), then summed in order
      R wv[(D + 1) * D];
#pragma unroll
      for (int i = 0; i < (D + 1) * D; ++i) wv[i] = We[(size_t)i * nd];
      int64_t vv[D + 1];
#pragma unroll
      for (int vl = 0; vl < D + 1; ++vl) vv[vl] = elem_verts[e * (D + 1) + vl];
      bool fr[D + 1];
#pragma unroll
      for (int vl = 0; vl < D + 1; ++vl) fr[vl] = vfree_of_lat[vv[vl]] >= 0;
      R xv[(D + 1) * D];
#pragma unroll
      for (int vl = 0; vl < D + 1; ++vl)
#pragma unroll
        for (int c = 0; c < D; ++c) xv[vl * D + c] = fr[vl] ? x0[vv[vl] * D + c] : R(0);
#pragma unroll
      for (int vl = 0; vl < D + 1; ++vl) {
        if (!fr[vl]) continue;
#pragma unroll
        for (int c = 0; c < D; ++c) acc += wv[vl * D + c] * xv[vl * D + c];
      }
    } else {
      for (int vl = 0; vl < nv; ++vl) {
        const int64_t v = elem_verts[e * nv + vl];
        if (vfree_of_lat[v] < 0) continue;
        for (int c = 0; c < d; ++c) acc += We[(size_t)(vl * d + c) * nd] * x0[v * d + c];
      }
    }
    y[idx] += acc;
  }
}

// E^d^T, facet part: fscr[g][v*d + c] = sum_q EF[g][q][v*d+c] r_F[q].  NFB > 0
// (= n_fb): a thread's n_fb entries and block values are loaded at once.
template <typename R, int NFB>
__global__ void k_edt_facet(SolveParams P, OpPtrs<R> O, const R* __restrict__ r, R* __restrict__ fscr) {
  const Sizes s = P.s;
  const int dd = s.d * s.d;
  const int64_t n = P.nff * dd;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t g = idx / dd;
    if (facet_off(P, g)) continue;
    int t = (int)(idx % dd);
    const R* E = O.EF + (size_t)g * s.nfb * dd + t;
    const R* rf = r + P.off_f + g * s.nfb;
    R acc = 0;
    if constexpr (NFB > 0) {
      R ev[NFB], rv[NFB];
#pragma unroll
      for (int q = 0; q < NFB; ++q) {
        ev[q] = E[(size_t)q * dd];
        rv[q] = rf[q];
      }
#pragma unroll
      for (int q = 0; q < NFB; ++q) acc += ev[q] * rv[q];
    } else {
      for (int q = 0; q < s.nfb; ++q) acc += E[(size_t)q * dd] * rf[q];
    }
    fscr[idx] = acc;
  }
}

// E^d^T, vertex part: b[lat(v)][c] = sum over incident (facet, slot) entries.
template <typename R>
__global__ void k_edt_vertex(int d, int64_t nfv, const int32_t* __restrict__ vinc_off, const int32_t* __restrict__ vinc,
                             const int32_t* __restrict__ free_to_lat, const R* __restrict__ fscr, R* __restrict__ b,
                             int compact) {
  const int dd = d * d;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nfv * d; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = idx / d;
    int c = (int)(idx % d);
    R acc = 0;
    // four incidences at a time: their index pairs, then their values, are
    // loaded together (the sum keeps its order)
    const int p0 = vinc_off[v], p1 = vinc_off[v + 1];
    int p = p0;
    for (; p + 4 <= p1; p += 4) {
      int2 iv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) iv[u] = make_int2(vinc[2 * (p + u)], vinc[2 * (p + u) + 1]);
      R fv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) fv[u] = fscr[(int64_t)iv[u].x * dd + iv[u].y * d + c];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += fv[u];
    }
    for (; p < p1; ++p) {
      int64_t g = vinc[2 * p];
      int sl = vinc[2 * p + 1];
      acc += fscr[g * dd + sl * d + c];
    }
    if (compact) b[idx] = acc;
    else b[(int64_t)free_to_lat[v] * d + c] = acc;
  }
}

// E^d: y_F (+)= sum_{v,c} EF[g][q][v*d+c] x[v][c]  (x lattice-indexed or compact).
// D > 0 (= d): the row of EF is loaded before the vertex ids.
template <typename R, int D>
__global__ void k_ed_facet(SolveParams P, OpPtrs<R> O, const int32_t* __restrict__ facet_vfree,
                           const int32_t* __restrict__ free_to_lat, const R* __restrict__ x0, R* __restrict__ y,
                           int add, int compact) {
  const Sizes s = P.s;
  const int d = D > 0 ? D : s.d, dd = d * d;
  const int64_t n = P.nff * s.nfb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t g = idx / s.nfb;
    if (facet_off(P, g)) continue;
    int q = (int)(idx % s.nfb);
    const R* E = O.EF + ((size_t)g * s.nfb + q) * dd;
    R acc = 0;
    if constexpr (D > 0) {
      R ev[D * D];
#pragma unroll
      for (int i = 0; i < D * D; ++i) ev[i] = E[i];
#pragma unroll
      for (int v = 0; v < D; ++v) {
        const int fv = facet_vfree[g * D + v];
        if (fv < 0) continue;
        const int64_t base = compact ? (int64_t)fv * D : (int64_t)free_to_lat[fv] * D;
#pragma unroll
        for (int c = 0; c < D; ++c) acc += ev[v * D + c] * x0[base + c];
      }
    } else {
      for (int v = 0; v < d; ++v) {
        int fv = facet_vfree[g * d + v];
        if (fv < 0) continue;
        int64_t base = compact ? (int64_t)fv * d : (int64_t)free_to_lat[fv] * d;
        for (int c = 0; c < d; ++c) acc += E[v * d + c] * x0[base + c];
      }
    }
    if (add) y[P.off_f + idx] += acc;
    else y[P.off_f + idx] = acc;
  }
}

// ---------------------------------------------------------------- multigrid
__device__ inline void mg_coords(int64_t v, const int* n, int c[3]) {
  int N0 = n[0] + 1, N1 = n[1] + 1;
  c[0] = (int)(v % N0);
  c[1] = (int)((v / N0) % N1);
  c[2] = (int)(v / ((int64_t)N0 * N1));
}

// Multigrid kernels run over the lattice blocks of a level, one block per
// blockIdx.y; vertex indices are block-local plus the block's offset.
// mode 0: x = Dinv b;  mode 1: r = b - A x;  mode 2: x += Dinv r (pointwise,
// r from a mode 1 launch: a Jacobi step never reads the x it writes), on the
// continuing blocks.  One 32-lane group per vertex, one stencil tap per lane.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_mg_point(MGLevelDev L, int mode) {
  constexpr int d = D, st = D == 3 ? 27 : 9, dd = D * D;
  const MGBlockDev B = load_block(L.blk + (blockIdx.y));
  if (L.active && !L.active[B.prob]) return;
  const R* A = (const R*)L.A;
  const R* Di = (const R*)L.Dinv;
  R* x = (R*)L.x;
  const R* b = (const R*)L.b;
  R* r = (R*)L.r;
  const int lane = threadIdx.x & 31;
  const int64_t gpb = blockDim.x >> 5;
  for (int64_t lv_ = blockIdx.x * gpb + (threadIdx.x >> 5); lv_ < B.nvert; lv_ += (int64_t)gridDim.x * gpb) {
    const int64_t v = B.voff + lv_;
    int c[3];
    mg_coords(lv_, B.n, c);
    const bool inner = lat_free(c, B.n, d, B.ffm);
    // the vertex's own values (lane 0) are loaded before the stencil products
    R bv[3] = {R(0), R(0), R(0)}, xv[3] = {R(0), R(0), R(0)}, Dv[9];
    if (lane == 0 && inner) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k < d) bv[k] = mode == 2 ? r[v * d + k] : b[v * d + k];
      if (mode != 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
          if (k < dd) Dv[k] = Di[(size_t)v * dd + k];
        if (mode == 2) {
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (k < d) xv[k] = x[v * d + k];
        }
      }
    }
    R part[3] = {R(0), R(0), R(0)};
    if (inner && mode == 1 && lane < st) {
      const int o = lane;
      int w[3] = {c[0] + o % 3 - 1, c[1] + (o / 3) % 3 - 1, d == 3 ? c[2] + o / 9 - 1 : 0};
      if (lat_free(w, B.n, d, B.ffm)) {
        const int64_t wi = B.voff + w[0] + (int64_t)(B.n[0] + 1) * (w[1] + (int64_t)(B.n[1] + 1) * w[2]);
        const R* Av = A + ((size_t)v * st + o) * dd;
        for (int k = 0; k < d; ++k)
          for (int m = 0; m < d; ++m) part[k] += Av[k * d + m] * x[wi * d + m];
      }
    }
    for (int k = 0; k < d; ++k) part[k] = group32_sum(part[k]);
    if (lane == 0) {
      if (!inner) {
        if (mode == 1)
          for (int k = 0; k < d; ++k) r[v * d + k] = R(0);
      } else {
        R res[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) res[k] = bv[k] - part[k];
        if (mode == 1) {
          for (int k = 0; k < d; ++k) r[v * d + k] = res[k];
        } else {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            if (k >= d) break;
            R u = R(0);
#pragma unroll
            for (int m = 0; m < 3; ++m)
              if (m < d) u += Dv[k * d + m] * res[m];
            x[v * d + k] = (mode == 0 ? R(0) : xv[k]) + u;
          }
        }
      }
    }
  }
}

__device__ inline int mg_cpos(int I, int n) { return (2 * I < n) ? 2 * I : n; }
__device__ inline double mg_w(int i, int I, int n) {
  int c = mg_cpos(I, n);
  if (i == c) return 1.0;
  bool is_coarse = (i % 2 == 0) || (i == n);
  if (!is_coarse && (i - c == 1 || c - i == 1)) return 0.5;
  return 0.0;
}

// b_c = P^T r_f (interior coarse vertices of each continuing block); one
// 32-lane group per coarse vertex.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_mg_restrict(MGLevelDev F, MGLevelDev C) {
  constexpr int d = D, st = D == 3 ? 27 : 9;
  const R* r = (const R*)F.r;
  R* bc = (R*)C.b;
  const MGBlockDev B = load_block(F.blk + (blockIdx.y));
  if (F.active && !F.active[B.prob]) return;
  const int lane = threadIdx.x & 31;
  const int64_t gpb = blockDim.x >> 5;
  for (int64_t V = blockIdx.x * gpb + (threadIdx.x >> 5); V < B.nvert_c; V += (int64_t)gridDim.x * gpb) {
    int CI[3];
    mg_coords(V, B.nc3, CI);
    const bool inner = lat_free(CI, B.nc3, d, B.ffm);
    R acc[3] = {R(0), R(0), R(0)};
    if (inner && lane < st) {
      const int o = lane;
      int base[3] = {mg_cpos(CI[0], B.n[0]), mg_cpos(CI[1], B.n[1]), d == 3 ? mg_cpos(CI[2], B.n[2]) : 0};
      int fi[3] = {base[0] + o % 3 - 1, base[1] + (o / 3) % 3 - 1, d == 3 ? base[2] + o / 9 - 1 : 0};
      if (lat_free(fi, B.n, d, B.ffm)) {
        double w = 1.0;
        for (int a = 0; a < d; ++a) w *= mg_w(fi[a], CI[a], B.n[a]);
        if (w != 0.0) {
          const int64_t fv = B.voff + fi[0] + (int64_t)(B.n[0] + 1) * (fi[1] + (int64_t)(B.n[1] + 1) * fi[2]);
          for (int k = 0; k < d; ++k) acc[k] = (R)w * r[fv * d + k];
        }
      }
    }
    for (int k = 0; k < d; ++k) acc[k] = group32_sum(acc[k]);
    if (lane == 0)
      for (int k = 0; k < d; ++k) bc[(B.cvoff + V) * d + k] = inner ? acc[k] : R(0);
  }
}

// x_f += P x_c (interior fine vertices of each continuing block); one 32-lane
// group per fine vertex, one candidate coarse vertex per lane.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_mg_prolong(MGLevelDev F, MGLevelDev C) {
  constexpr int d = D, st = D == 3 ? 27 : 9;
  R* x = (R*)F.x;
  const R* xc = (const R*)C.x;
  const MGBlockDev B = load_block(F.blk + (blockIdx.y));
  if (F.active && !F.active[B.prob]) return;
  const int lane = threadIdx.x & 31;
  const int64_t gpb = blockDim.x >> 5;
  for (int64_t lv_ = blockIdx.x * gpb + (threadIdx.x >> 5); lv_ < B.nvert; lv_ += (int64_t)gridDim.x * gpb) {
    int fi[3];
    mg_coords(lv_, B.n, fi);
    const bool inner = lat_free(fi, B.n, d, B.ffm);
    R acc[3] = {R(0), R(0), R(0)};
    if (inner && lane < st) {
      const int o = lane;
      int CI[3] = {fi[0] / 2 - 1 + o % 3, fi[1] / 2 - 1 + (o / 3) % 3, d == 3 ? fi[2] / 2 - 1 + o / 9 : 0};
      bool ok = true;
      for (int a = 0; a < d; ++a)
        if (CI[a] < 0 || CI[a] > B.nc3[a]) ok = false;
      if (ok && lat_free(CI, B.nc3, d, B.ffm)) {
        double w = 1.0;
        for (int a = 0; a < d; ++a) w *= mg_w(fi[a], CI[a], B.n[a]);
        if (w != 0.0) {
          const int64_t cv = B.cvoff + CI[0] + (int64_t)(B.nc3[0] + 1) * (CI[1] + (int64_t)(B.nc3[1] + 1) * CI[2]);
          for (int k = 0; k < d; ++k) acc[k] = (R)w * xc[cv * d + k];
        }
      }
    }
    for (int k = 0; k < d; ++k) acc[k] = group32_sum(acc[k]);
    if (lane == 0 && inner)
      for (int k = 0; k < d; ++k) x[(B.voff + lv_) * d + k] += acc[k];
  }
}

// Coarsest blocks of a level: x = C^{-1} b over each block's free dofs (FP64
// accumulation), one wave per row of the (symmetric) inverse; blockIdx.y runs
// over the level's coarsest blocks.
template <typename R>
__global__ void k_mg_coarse(const double* __restrict__ Cinv_all, const int32_t* __restrict__ cmap_all, int d,
                            MGLevelDev L) {
  const R* b = (const R*)L.b;
  R* x = (R*)L.x;
  const MGBlockDev B = load_block(L.blk + (L.ncont + blockIdx.y));
  if (L.active && !L.active[B.prob]) return;
  const int64_t nc = B.nc, o = B.voff * d;
  const double* Cinv = Cinv_all + B.cinv_off;
  const int32_t* cmap = cmap_all + B.cmap_off;
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  for (int64_t i = blockIdx.x * wpb + (threadIdx.x >> 6); i < nc; i += (int64_t)gridDim.x * wpb) {
    double acc = 0.0;
    for (int64_t j = lane; j < nc; j += 64) acc += Cinv[i * nc + j] * (double)b[o + cmap[j]];
    acc = wave_sum(acc);
    if (lane == 0) x[o + cmap[i]] = (R)acc;
  }
}

// ------------------------------------------------------------ pressure parts
// y_p = M_p^{-1} (r_p - B a) with M_p^{-1} = (nu_T/|det J|) Mp^-1_ref; the
// velocity is gathered once (scaled by the Piola factors of B), then each
// wave reduces one pressure row at a time.
template <typename R>
__global__ void __launch_bounds__(256) k_elem_press(SolveParams P, const R* __restrict__ a, const R* __restrict__ r,
                                                    R* __restrict__ y, int with_B) {
  const Sizes s = P.s;
  const int nb = s.nb, nd = s.nd, np = s.np, nu = s.nu;
  __shared__ double us[MAXNB + MAXND];
  __shared__ double bp[MAXNP];
  __shared__ int rmap[MAXNB + MAXND];
  __shared__ R ad[MAXND], ab[MAXNB];
  __shared__ double rp[MAXNP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  build_rowmap(s, rmap);
  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    if (elem_off(P, e)) continue;
    const double det = P.detJ[e];
    const double nue = P.nu[e];
    // the element's own values are loaded with the facet ids, ahead of the
    // facet values that depend on them
    if (tid < np) rp[tid] = (double)r[P.off_p + e * np + tid];
    if (with_B) {
      const double sb = -fabs(det), sf = det > 0 ? -1.0 : 1.0;
      if (tid < nb) ab[tid] = a[e * nb + tid];
      gather_elem_d(P, a, e, ad);
      __syncthreads();
      for (int row = tid; row < nb + nd; row += blockDim.x) {
        int iu = rmap[row];
        if (iu >= 0) us[iu] = (row < nb ? sb * (double)ab[row] : sf * (double)ad[row - nb]);
      }
    }
    __syncthreads();
    if (with_B) {
      bu_rows(P.rBp, nu, np, us, wave, lane, [&](int q, double a) { bp[q] = rp[q] - a; });
    } else {
      for (int q = tid; q < np; q += blockDim.x) bp[q] = rp[q];
    }
    __syncthreads();
    if (tid < np) {
      double sc = nue / fabs(det);
      const double acc = dot_strided8(P.rMpinv + (size_t)tid * np, 1, bp, np);
      y[P.off_p + e * np + tid] = (R)(sc * acc);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ point values
// u and p of a solution x at barycentric points given w.r.t. each element's
// vertices in the caller's order (pts [npts][nv]); one workgroup per element,
// one thread per point.  Velocity basis (sorted vertices, J = [x_j - x_0]):
// bubbles lambda^alpha J w, facet functions lambda^beta J w / det J (w the
// reference vector of the function, rphi); pressure lambda^gamma.
__global__ void k_eval(SolveParams P, const double* __restrict__ coords, const int32_t* __restrict__ elem_verts,
                       const int32_t* __restrict__ elem_perm, const double* __restrict__ rphi,
                       const double* __restrict__ rpidx, int npts, const double* __restrict__ pts,
                       const double* __restrict__ x, double* __restrict__ u, double* __restrict__ p) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1;
  for (int64_t e = blockIdx.x; e < P.ne; e += gridDim.x) {
    // caller order of the sorted vertices: decode the permutation rank
    int perm[4], avail[4];
    {
      int r = elem_perm[e], dig[4];
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
    double X[4][3], J[3][3];
    for (int j = 0; j < nv; ++j) {
      const int v = elem_verts[e * nv + j];
      for (int r = 0; r < 3; ++r) X[j][r] = r < d ? coords[(size_t)v * d + r] : 0.0;
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] = (r < d && c < d) ? X[c + 1][r] - X[0][r] : 0.0;
    const double idet = 1.0 / P.detJ[e];
    for (int q = threadIdx.x; q < npts; q += blockDim.x) {
      double lam[4];
      for (int j = 0; j < nv; ++j) lam[j] = pts[q * nv + perm[j]];
      double uv[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < s.nu; ++i) {
        double c;
        if (i < s.nb) {
          c = x[e * s.nb + i];
        } else {
          const int f = (i - s.nb) / s.nF, qq = (i - s.nb) % s.nF;
          const int g = P.elem_ff[e * nv + f];
          c = g >= 0 ? x[P.off_f + (int64_t)g * s.nfb + qq] * idet
                     : (P.xD ? P.xD[e * s.nd + f * s.nfb + qq] * idet : 0.0);
        }
        if (c == 0.0) continue;
        const double* ph = rphi + (size_t)i * (nv + 3);
        double m = 1.0;
        for (int j = 0; j < nv; ++j)
          for (int t = 0; t < (int)ph[j]; ++t) m *= lam[j];
        for (int r = 0; r < d; ++r) {
          double jw = 0.0;
          for (int cc = 0; cc < d; ++cc) jw += J[r][cc] * ph[nv + cc];
          uv[r] += c * m * jw;
        }
      }
      double pv = 0.0;
      for (int g = 0; g < s.np; ++g) {
        double m = 1.0;
        for (int j = 0; j < nv; ++j)
          for (int t = 0; t < (int)rpidx[g * nv + j]; ++t) m *= lam[j];
        pv += x[P.off_p + e * s.np + g] * m;
      }
      for (int r = 0; r < d; ++r) u[((size_t)e * npts + q) * d + r] = uv[r];
      p[(size_t)e * npts + q] = pv;
    }
  }
}

void launch_eval(hipStream_t st, const SolveParams& P, const double* coords, const int32_t* elem_verts,
                 const int32_t* elem_perm, const double* rphi, const double* rpidx, int npts, const double* pts,
                 const double* x, double* u, double* p) {
  hipLaunchKernelGGL(k_eval, dim3((unsigned)std::min<int64_t>(P.ne, 1 << 20)), dim3(64), 0, st, P, coords,
                     elem_verts, elem_perm, rphi, rpidx, npts, pts, x, u, p);
}

// ----------------------------------------------------------------- vectors
template <typename R>
__global__ void k_axpby(int64_t n, double a, const R* __restrict__ x, double b, R* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (R)(a * (double)x[i] + (b == 0.0 ? 0.0 : b * (double)y[i]));
}

template <typename R>
__global__ void k_fill(int64_t n, R v, R* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = v;
}

template <typename A, typename B>
__global__ void k_convert(int64_t n, const A* __restrict__ x, B* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = (B)x[i];
}

// Deterministic two-stage dot product: partial sums per block, FP64.
template <typename R>
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const R* __restrict__ x, const R* __restrict__ y,
                                                     double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_partials(int n, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// MINRES direction / iterate update: w_new = a v + b w1 + c w2 (stored in w1), x += phi w_new.
template <typename R>
__global__ void k_minres_w(int64_t n, const R* __restrict__ v, R* __restrict__ w1, const R* __restrict__ w2,
                           R* __restrict__ x, double a, double b, double c, double phi) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double wn = a * (double)v[i] + b * (double)w1[i] + c * (double)w2[i];
    w1[i] = (R)wn;
    x[i] = (R)((double)x[i] + phi * wn);
  }
}

// y (double) += a * x (R)  /  y (B) = a * x (A)
template <typename A, typename B>
__global__ void k_scale_convert(int64_t n, double a, const A* __restrict__ x, B* __restrict__ y, int add) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * (double)x[i];
    y[i] = add ? (B)((double)y[i] + v) : (B)v;
  }
}

// compact P1 vector (free vertices) <-> lattice-indexed vector
template <typename R>
__global__ void k_scatter_compact(int64_t nfv, int d, const int32_t* __restrict__ f2l, const R* __restrict__ c,
                                  R* __restrict__ lat) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nfv * d; i += (int64_t)gridDim.x * blockDim.x)
    lat[(int64_t)f2l[i / d] * d + i % d] = c[i];
}
template <typename R>
__global__ void k_gather_compact(int64_t nfv, int d, const int32_t* __restrict__ f2l, const R* __restrict__ lat,
                                 R* __restrict__ c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nfv * d; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = lat[(int64_t)f2l[i / d] * d + i % d];
}

// ------------------------------------------------------------------ launchers
// ------------------------------------------------ full-system variant (FP64)
// One colour phase of overlapping block Gauss-Seidel on A (Theorem aux_pc,
// Corollary aux_pc_mult): per block (a facet with its free dofs and the
// bubbles of its neighbours) r_B = s_B - (A x)_B from the maintained element
// products y_T = A_T x_T, x_B += D_B^{-1} r_B, then y_T += A_T[:, B] delta for
// both neighbours.  Blocks of one colour share no element.
__device__ inline int64_t full_dof(const SolveParams& P, const FullDev& F, int nf, int g, int64_t e0, int64_t e1,
                                   int j) {
  const Sizes& s = P.s;
  if (j < nf) return P.off_f + (int64_t)g * s.nfb + j;
  if (j < nf + s.nb) return e0 * s.nb + (j - nf);
  return e1 * s.nb + (j - nf - s.nb);
}

__global__ void __launch_bounds__(256) k_full_smooth(SolveParams P, FullDev F, int c0, int c1, double* __restrict__ x,
                                                     const double* __restrict__ sv, double* __restrict__ y) {
  const Sizes s = P.s;
  const int nA = s.nA, nb = s.nb, nfb = s.nfb, nbk = F.nbk, tid = threadIdx.x;
  __shared__ double r[64], dl[64];
  for (int64_t i = c0 + blockIdx.x; i < c1; i += gridDim.x) {
    const int64_t b = F.colour_blocks[i];
    const int64_t e0 = F.blk_el[2 * b], e1 = F.blk_el[2 * b + 1];
    const int s0 = F.blk_slot[2 * b], s1 = F.blk_slot[2 * b + 1];
    const int g = F.blk_g[b];
    const int nside = e1 >= 0 ? 2 : 1;
    const int nf = g >= 0 ? nfb : 0;
    const int m = nf + nb * nside;
    if (tid < m) {
      double yy;
      if (tid < nf) yy = y[e0 * nA + nb + s0 * nfb + tid] + (e1 >= 0 ? y[e1 * nA + nb + s1 * nfb + tid] : 0.0);
      else if (tid < nf + nb) yy = y[e0 * nA + tid - nf];
      else yy = y[e1 * nA + tid - nf - nb];
      r[tid] = sv[full_dof(P, F, nf, g, e0, e1, tid)] - yy;
    }
    __syncthreads();
    if (tid < m) {
      const double* Bi = F.Binv + (size_t)b * nbk * nbk + tid;   // symmetric: column tid
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += Bi[(size_t)j * nbk] * r[j];
      dl[tid] = acc;
      x[full_dof(P, F, nf, g, e0, e1, tid)] += acc;
    }
    __syncthreads();
    for (int t = tid; t < nside * nA; t += blockDim.x) {
      const int side = t / nA, row = t % nA;
      const int64_t e = side ? e1 : e0;
      const int sl = side ? s1 : s0;
      const double* Ae = F.A + (size_t)e * nA * nA + row;   // A_T symmetric: rows as columns
      double acc = 0.0;
      for (int q = 0; q < nf; ++q) acc += Ae[(size_t)(nb + sl * nfb + q) * nA] * dl[q];
      const int o = nf + side * nb;
      for (int j = 0; j < nb; ++j) acc += Ae[(size_t)j * nA] * dl[o + j];
      y[e * nA + row] += acc;
    }
    __syncthreads();
  }
}

// r = s - A x on the velocity dofs, from the maintained products.
__global__ void k_full_resid(SolveParams P, int nA, const double* __restrict__ sv, const double* __restrict__ y,
                             double* __restrict__ r) {
  const Sizes s = P.s;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < P.off_p;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double yy;
    if (idx < P.off_f) {
      yy = y[(idx / s.nb) * nA + idx % s.nb];
    } else {
      const int64_t g = (idx - P.off_f) / s.nfb;
      const int q = (int)((idx - P.off_f) % s.nfb);
      yy = y[(int64_t)P.facet_el[2 * g] * nA + s.nb + P.facet_slot[2 * g] * s.nfb + q];
      if (P.facet_el[2 * g + 1] >= 0) yy += y[(int64_t)P.facet_el[2 * g + 1] * nA + s.nb + P.facet_slot[2 * g + 1] * s.nfb + q];
    }
    r[idx] = sv[idx] - yy;
  }
}

// E^T, bubble rows: eto[e][m] = sum_i Eo[e][i][m] r_o,e[i].
__global__ void k_full_edt(SolveParams P, FullDev F, const double* __restrict__ r, double* __restrict__ eto) {
  const Sizes s = P.s;
  const int nvd = (s.d + 1) * s.d;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < P.ne * nvd;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / nvd;
    const int m = (int)(idx % nvd);
    const double* E = F.Eo + (size_t)e * s.nb * nvd + m;
    double acc = 0.0;
    for (int i = 0; i < s.nb; ++i) acc += E[(size_t)i * nvd] * r[e * s.nb + i];
    eto[idx] = acc;
  }
}

// b[v][c] += sum over the elements at lattice vertex v of eto[e][vl*d + c]
// (free vertices only; fixed order).
__global__ void k_full_edt_vertex(int d, int64_t nvert, const int32_t* __restrict__ vert_elem_off,
                                  const int32_t* __restrict__ vert_elem, const int32_t* __restrict__ elem_verts,
                                  const int32_t* __restrict__ vfree_of_lat, const double* __restrict__ eto,
                                  double* __restrict__ b) {
  const int nv = d + 1, nvd = nv * d;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nvert * d;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = idx / d;
    const int c = (int)(idx % d);
    if (vfree_of_lat[v] < 0) continue;
    double acc = 0.0;
    for (int p = vert_elem_off[v]; p < vert_elem_off[v + 1]; ++p) {
      const int64_t e = vert_elem[p];
      for (int vl = 0; vl < nv; ++vl)
        if (elem_verts[e * nv + vl] == v) acc += eto[e * nvd + vl * d + c];
    }
    b[idx] += acc;
  }
}

// E, bubble rows: x_o,e[i] += sum_{vl,c} Eo[e][i][vl*d + c] x0[v][c].
__global__ void k_full_ed(SolveParams P, FullDev F, const int32_t* __restrict__ elem_verts,
                          const int32_t* __restrict__ vfree_of_lat, const double* __restrict__ x0,
                          double* __restrict__ x) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1, nvd = nv * d;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < P.ne * s.nb;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / s.nb;
    const double* E = F.Eo + (size_t)idx * nvd;
    double acc = 0.0;
    for (int vl = 0; vl < nv; ++vl) {
      const int64_t v = elem_verts[e * nv + vl];
      if (vfree_of_lat[v] < 0) continue;
      for (int c = 0; c < d; ++c) acc += E[vl * d + c] * x0[v * d + c];
    }
    x[idx] += acc;
  }
}

// y_T += W_T x0_T after the coarse correction (W_T = A_T E_T).
__global__ void k_full_ycorr(SolveParams P, FullDev F, const int32_t* __restrict__ elem_verts,
                             const int32_t* __restrict__ vfree_of_lat, const double* __restrict__ x0,
                             double* __restrict__ y) {
  const Sizes s = P.s;
  const int d = s.d, nv = d + 1, nvd = nv * d, nA = s.nA;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < P.ne * nA;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / nA;
    const int t = (int)(idx % nA);
    const double* We = F.W + (size_t)e * nvd * nA + t;
    double acc = 0.0;
    for (int vl = 0; vl < nv; ++vl) {
      const int64_t v = elem_verts[e * nv + vl];
      if (vfree_of_lat[v] < 0) continue;
      for (int c = 0; c < d; ++c) acc += We[(size_t)(vl * d + c) * nA] * x0[v * d + c];
    }
    y[idx] += acc;
  }
}

static int grid_for(int64_t n, int per = 256) {
  int64_t g = (n + per - 1) / per;
  if (g > 65535 * 8) g = 65535 * 8;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_full_smooth(hipStream_t st, const SolveParams& P, const FullDev& F, int c0, int c1, double* x,
                        const double* sv, double* y) {
  if (c1 <= c0) return;
  hipLaunchKernelGGL(k_full_smooth, dim3((unsigned)std::min(c1 - c0, 1 << 20)), dim3(256), 0, st, P, F, c0, c1, x, sv, y);
}
void launch_full_resid(hipStream_t st, const SolveParams& P, const double* sv, const double* y, double* r) {
  hipLaunchKernelGGL(k_full_resid, dim3(grid_for(P.off_p)), dim3(256), 0, st, P, P.s.nA, sv, y, r);
}
void launch_full_edt(hipStream_t st, const SolveParams& P, const FullDev& F, const double* r, double* eto,
                     int64_t nvert, const int32_t* vert_elem_off, const int32_t* vert_elem, const int32_t* elem_verts,
                     const int32_t* vfree_of_lat, double* b) {
  const int d = P.s.d;
  hipLaunchKernelGGL(k_full_edt, dim3(grid_for(P.ne * (d + 1) * d)), dim3(256), 0, st, P, F, r, eto);
  hipLaunchKernelGGL(k_full_edt_vertex, dim3(grid_for(nvert * d)), dim3(256), 0, st, d, nvert, vert_elem_off, vert_elem,
                     elem_verts, vfree_of_lat, eto, b);
}
void launch_full_ed(hipStream_t st, const SolveParams& P, const FullDev& F, const int32_t* elem_verts,
                    const int32_t* vfree_of_lat, const double* x0, double* x, double* y) {
  hipLaunchKernelGGL(k_full_ed, dim3(grid_for(P.ne * P.s.nb)), dim3(256), 0, st, P, F, elem_verts, vfree_of_lat, x0, x);
  hipLaunchKernelGGL(k_full_ycorr, dim3(grid_for(P.ne * P.s.nA)), dim3(256), 0, st, P, F, elem_verts, vfree_of_lat, x0,
                     y);
}
static int elem_grid(int64_t ne) { return (int)std::min<int64_t>(ne, 1 << 20); }

template <typename R, typename MA>
static void elem_apply_launch(hipStream_t st, const SolveParams& P, MA Ad, MA H, MA Aoo, const R* x, R* y, R* escr,
                              int flags) {
  // the operator apply K x and the B^T-only apply of K-hat^{-1} run every
  // MINRES iteration: compile-time flags for them; K x with plain storage and
  // even n_d takes two rows of A^d per thread
  const dim3 g(elem_grid(P.ne)), b(256);
  if constexpr (std::is_same<MA, MatP<R>>::value) {
    // H read once through LDS when its rows fit 64 KiB (k <= 4)
    const int ldh = P.s.nd | 1;
    const size_t hb = (size_t)P.s.nb * ldh * sizeof(R);
    const int hl = hb <= 65536 ? ldh : 0;
    const size_t lds = hl ? hb : 0;
    const int rpt = P.apply_rpt;   // 0: the largest the sizes allow
    // FP32 with n_d divisible by 4: four rows per thread (16-byte loads)
    if constexpr (sizeof(R) == 4) {
      if (flags == (1 | 2 | 4) && P.s.nd % 4 == 0 && (rpt == 0 || rpt == 4)) {
        hipLaunchKernelGGL((k_elem_apply<R, MA, 7, 4>), g, b, lds, st, P, Ad, H, Aoo, x, y, escr, flags, hl);
        return;
      }
    }
    if (flags == (1 | 2 | 4) && P.s.nd % 2 == 0 && rpt != 1) {
      hipLaunchKernelGGL((k_elem_apply<R, MA, 7, 2>), g, b, lds, st, P, Ad, H, Aoo, x, y, escr, flags, hl);
      return;
    }
  }
  if (flags == (1 | 2 | 4))
    hipLaunchKernelGGL((k_elem_apply<R, MA, 7, 1>), g, b, 0, st, P, Ad, H, Aoo, x, y, escr, flags, 0);
  else if (flags == (2 | 16))
    hipLaunchKernelGGL((k_elem_apply<R, MA, 18, 1>), g, b, 0, st, P, Ad, H, Aoo, x, y, escr, flags, 0);
  else
    hipLaunchKernelGGL((k_elem_apply<R, MA, -1, 1>), g, b, 0, st, P, Ad, H, Aoo, x, y, escr, flags, 0);
}
// Whether the A^d product of k_elem_apply with cp rows per thread splits the
// columns over two waves (its sums then differ in rounding from the unsplit ones).
bool apply_col_split(int nd, int cp) { return cp == 4 && nd > 0; }
// Lanes per row of H in z_o = x_o + H x_d of k_elem_apply with cp rows of
// A^d per thread (the split of the 256 threads above): rows are summed in
// lane-strided order, so choices of cp with the same width give bitwise the
// same results, and choices with different widths differ in rounding only.
int apply_h_lanes(int nd, int cp) {
  const int tA = apply_col_split(nd, cp) ? 128 : ((nd / cp + 63) >> 6) << 6;
  if (tA >= 256) return 16;
  return 256 - tA >= 128 ? 16 : 4;
}
template <typename R>
void launch_elem_apply(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* x, R* y, R* escr, int flags) {
  if constexpr (sizeof(R) == 8) {
    if (!O.Ad) {   // split storage: FP64 entries as FP32 hi + lo
      elem_apply_launch<R, MatHL>(st, P, MatHL{O.hAd, O.lAd}, MatHL{O.hH, O.lH}, MatHL{O.hAoo, O.lAoo}, x, y, escr, flags);
      return;
    }
  }
  elem_apply_launch<R, MatP<R>>(st, P, MatP<R>{O.Ad}, MatP<R>{O.H}, MatP<R>{O.Aoo}, x, y, escr, flags);
}
template <typename R>
void launch_facet_sum(hipStream_t st, const SolveParams& P, const R* escr, const R* base, R sign, R* y) {
  hipLaunchKernelGGL(k_facet_sum<R>, dim3(grid_for(P.nff * P.s.nfb)), dim3(256), 0, st, P, escr, base, sign, y);
}
template <typename R>
void launch_ext_pre(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* r, R* to, R* escr) {
  if (P.s.nb <= 24 && P.s.nd + P.s.nb <= 256)
    hipLaunchKernelGGL((k_ext_pre<R, 24>), dim3(elem_grid(P.ne)), dim3(256), 0, st, P, O, r, to, escr);
  else
    hipLaunchKernelGGL((k_ext_pre<R, 0>), dim3(elem_grid(P.ne)), dim3(256), 0, st, P, O, r, to, escr);
}
template <typename R>
void launch_ext_post(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* t, const R* to, R* y) {
  if (P.s.nb <= 32 && P.s.nd <= 96)
    hipLaunchKernelGGL((k_ext_post<R, 12, 1>), dim3(elem_grid(P.ne)), dim3(256), 0, st, P, O, t, to, y);
  else if (P.s.nb <= 64 && P.s.nd <= 144)
    hipLaunchKernelGGL((k_ext_post<R, 18, 2>), dim3(elem_grid(P.ne)), dim3(256), 0, st, P, O, t, to, y);
  else
    hipLaunchKernelGGL((k_ext_post<R, 0, 1>), dim3(elem_grid(P.ne)), dim3(256), 0, st, P, O, t, to, y);
}
// facets_per_block (1 or 2) and grid_cap choose the launch shape; every
// shape gives the same result.
template <typename R, int NFB>
static void smooth_launch(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, int32_t c0, int32_t c1, R* x,
                          const R* s, R* y, int fpw, int64_t cap, int T1) {
  // two teams per workgroup only for facet blocks up to 22 (LDS of the
  // double-buffered D_F^{-1})
  if constexpr (NFB > 22) fpw = 1;
  const int64_t blocks = std::min<int64_t>((c1 - c0 + fpw - 1) / fpw, cap);
  if constexpr (NFB <= 22) {
    if (fpw == 2) {
      if (P.has_outlet)
        hipLaunchKernelGGL((k_smooth_y<R, NFB, 2, true>), dim3((unsigned)blocks), dim3(2 * T1), 0, st, P, O, c0, c1, x,
                           s, y, T1);
      else
        hipLaunchKernelGGL((k_smooth_y<R, NFB, 2, false>), dim3((unsigned)blocks), dim3(2 * T1), 0, st, P, O, c0, c1,
                           x, s, y, T1);
      return;
    }
  }
  if constexpr (NFB == 6 || NFB == 12 || NFB == 22 || (NFB == 35 && sizeof(R) == 4)) {
    // 3D: two columns per thread
    if (P.s.nd == 4 * NFB && P.s.d == 3) {
      const unsigned b2 = (unsigned)std::min<int64_t>(c1 - c0, cap);
      constexpr int T2 = ((4 * NFB + 63) / 64) * 64;
      if (P.has_outlet)
        hipLaunchKernelGGL((k_smooth_y2<R, NFB, true>), dim3(b2), dim3(T2), 0, st, P, O, c0, c1, x, s, y);
      else
        hipLaunchKernelGGL((k_smooth_y2<R, NFB, false>), dim3(b2), dim3(T2), 0, st, P, O, c0, c1, x, s, y);
      return;
    }
  }
  if (P.has_outlet)
    hipLaunchKernelGGL((k_smooth_y<R, NFB, 1, true>), dim3((unsigned)blocks), dim3(T1), 0, st, P, O, c0, c1, x, s, y,
                       T1);
  else
    hipLaunchKernelGGL((k_smooth_y<R, NFB, 1, false>), dim3((unsigned)blocks), dim3(T1), 0, st, P, O, c0, c1, x, s, y,
                       T1);
}
int smooth_team_threads(int nd) { return ((2 * nd + 63) / 64) * 64; }
template <typename R>
void launch_smooth_phase(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, int32_t c0, int32_t c1, R* x,
                         const R* s, R* y, int fpw, int64_t cap) {
  if (c1 <= c0) return;
  const int T1 = smooth_team_threads(P.s.nd);
  if (fpw != 2 || 2 * T1 > 512) fpw = 1;
  if (cap <= 0) cap = 1 << 20;
  switch (P.s.nfb) {
    case 5: smooth_launch<R, 5>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 6: smooth_launch<R, 6>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 7: smooth_launch<R, 7>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 9: smooth_launch<R, 9>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 11: smooth_launch<R, 11>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 12: smooth_launch<R, 12>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 22: smooth_launch<R, 22>(st, P, O, c0, c1, x, s, y, fpw, cap, T1); break;
    case 35: smooth_launch<R, 35>(st, P, O, c0, c1, x, s, y, 1, cap, T1); break;
    case 51: smooth_launch<R, 51>(st, P, O, c0, c1, x, s, y, 1, cap, T1); break;
    default: break;
  }
}
template <typename R, int NFB>
static void smooth_last_launch(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, int32_t c0, int32_t c1, R* x,
                               const R* s, const R* y) {
  const dim3 g(grid_for((int64_t)(c1 - c0) * NFB)), b(256);
  if (P.has_outlet)
    hipLaunchKernelGGL((k_smooth_last<R, NFB, true>), g, b, 0, st, P, O, c0, c1, x, s, y);
  else
    hipLaunchKernelGGL((k_smooth_last<R, NFB, false>), g, b, 0, st, P, O, c0, c1, x, s, y);
}
template <typename R>
void launch_smooth_last(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, int32_t c0, int32_t c1, R* x,
                        const R* s, const R* y) {
  if (c1 <= c0) return;
  switch (P.s.nfb) {
    case 5: smooth_last_launch<R, 5>(st, P, O, c0, c1, x, s, y); break;
    case 6: smooth_last_launch<R, 6>(st, P, O, c0, c1, x, s, y); break;
    case 7: smooth_last_launch<R, 7>(st, P, O, c0, c1, x, s, y); break;
    case 9: smooth_last_launch<R, 9>(st, P, O, c0, c1, x, s, y); break;
    case 11: smooth_last_launch<R, 11>(st, P, O, c0, c1, x, s, y); break;
    case 12: smooth_last_launch<R, 12>(st, P, O, c0, c1, x, s, y); break;
    case 22: smooth_last_launch<R, 22>(st, P, O, c0, c1, x, s, y); break;
    case 35: smooth_last_launch<R, 35>(st, P, O, c0, c1, x, s, y); break;
    case 51: smooth_last_launch<R, 51>(st, P, O, c0, c1, x, s, y); break;
    default: break;
  }
}
template <typename R>
void launch_block_jacobi(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* r, R* z) {
  hipLaunchKernelGGL(k_block_jacobi<R>, dim3(grid_for(P.nff * P.s.nfb)), dim3(256), 0, st, P, O, r, z);
}
template <typename R>
void launch_ycorr(hipStream_t st, const SolveParams& P, const R* W, const int32_t* elem_verts,
                  const int32_t* vfree_of_lat, const R* x0, R* y) {
  const dim3 ge(grid_for(P.ne * P.s.nd)), be(256);
  if (P.s.d == 3)
    hipLaunchKernelGGL((k_elem_ycorr<R, 3>), ge, be, 0, st, P, W, elem_verts, vfree_of_lat, x0, y);
  else
    hipLaunchKernelGGL((k_elem_ycorr<R, 0>), ge, be, 0, st, P, W, elem_verts, vfree_of_lat, x0, y);
}
template <typename R>
void launch_edt(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* r, R* fscr, int64_t nfv,
                const int32_t* vinc_off, const int32_t* vinc, const int32_t* free_to_lat, R* b, int compact) {
  const dim3 ge(grid_for(P.nff * P.s.d * P.s.d)), be(256);
  switch (P.s.nfb) {
    case 12: hipLaunchKernelGGL((k_edt_facet<R, 12>), ge, be, 0, st, P, O, r, fscr); break;
    case 22: hipLaunchKernelGGL((k_edt_facet<R, 22>), ge, be, 0, st, P, O, r, fscr); break;
    case 35: hipLaunchKernelGGL((k_edt_facet<R, 35>), ge, be, 0, st, P, O, r, fscr); break;
    default: hipLaunchKernelGGL((k_edt_facet<R, 0>), ge, be, 0, st, P, O, r, fscr); break;
  }
  hipLaunchKernelGGL(k_edt_vertex<R>, dim3(grid_for(nfv * P.s.d)), dim3(256), 0, st, P.s.d, nfv, vinc_off, vinc,
                     free_to_lat, (const R*)fscr, b, compact);
}
template <typename R>
void launch_ed(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const int32_t* facet_vfree,
               const int32_t* free_to_lat, const R* x0, R* y, int add, int compact) {
  const dim3 ge(grid_for(P.nff * P.s.nfb)), be(256);
  if (P.s.d == 3)
    hipLaunchKernelGGL((k_ed_facet<R, 3>), ge, be, 0, st, P, O, facet_vfree, free_to_lat, x0, y, add, compact);
  else
    hipLaunchKernelGGL((k_ed_facet<R, 0>), ge, be, 0, st, P, O, facet_vfree, free_to_lat, x0, y, add, compact);
}
static unsigned mg_grid(int64_t n, int per) {
  int64_t g = (n + per - 1) / per;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}
template <typename R>
void launch_mg_point(hipStream_t st, int d, const MGLevelDev& L, int mode) {
  if (L.ncont == 0) return;
  const dim3 g(mg_grid(L.maxv, 8), L.ncont), b(256);
  if (d == 3)
    hipLaunchKernelGGL((k_mg_point<R, 3>), g, b, 0, st, L, mode);
  else
    hipLaunchKernelGGL((k_mg_point<R, 2>), g, b, 0, st, L, mode);
}
template <typename R>
void launch_mg_restrict(hipStream_t st, int d, const MGLevelDev& F, const MGLevelDev& C) {
  if (F.ncont == 0) return;
  const dim3 g(mg_grid(F.maxvc, 8), F.ncont), b(256);
  if (d == 3)
    hipLaunchKernelGGL((k_mg_restrict<R, 3>), g, b, 0, st, F, C);
  else
    hipLaunchKernelGGL((k_mg_restrict<R, 2>), g, b, 0, st, F, C);
}
template <typename R>
void launch_mg_prolong(hipStream_t st, int d, const MGLevelDev& F, const MGLevelDev& C) {
  if (F.ncont == 0) return;
  const dim3 g(mg_grid(F.maxv, 8), F.ncont), b(256);
  if (d == 3)
    hipLaunchKernelGGL((k_mg_prolong<R, 3>), g, b, 0, st, F, C);
  else
    hipLaunchKernelGGL((k_mg_prolong<R, 2>), g, b, 0, st, F, C);
}
template <typename R>
void launch_mg_coarse(hipStream_t st, const double* Cinv, const int32_t* cmap, int d, const MGLevelDev& L) {
  const int nco = L.nblk - L.ncont;
  if (nco == 0) return;
  hipLaunchKernelGGL(k_mg_coarse<R>, dim3(mg_grid(L.maxnc, 4), nco), dim3(256), 0, st, Cinv, cmap, d, L);
}
template <typename R>
void launch_elem_press(hipStream_t st, const SolveParams& P, const R* a, const R* r, R* y, int with_B) {
  hipLaunchKernelGGL(k_elem_press<R>, dim3(elem_grid(P.ne)), dim3(256), 0, st, P, a, r, y, with_B);
}
template <typename R>
void launch_axpby(hipStream_t st, int64_t n, double a, const R* x, double b, R* y) {
  hipLaunchKernelGGL(k_axpby<R>, dim3(grid_for(n)), dim3(256), 0, st, n, a, x, b, y);
}
template <typename R>
void launch_fill(hipStream_t st, int64_t n, R v, R* y) {
  hipLaunchKernelGGL(k_fill<R>, dim3(grid_for(n)), dim3(256), 0, st, n, v, y);
}
template <typename A, typename B>
void launch_convert(hipStream_t st, int64_t n, const A* x, B* y) {
  hipLaunchKernelGGL((k_convert<A, B>), dim3(grid_for(n)), dim3(256), 0, st, n, x, y);
}
template <typename R>
void launch_dot(hipStream_t st, int64_t n, const R* x, const R* y, double* part, double* out) {
  int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_dot_partial<R>, dim3(nb), dim3(256), 0, st, n, x, y, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, nb, (const double*)part, out);
}

template <typename R>
void launch_scatter_compact(hipStream_t st, int64_t nfv, int d, const int32_t* f2l, const R* c, R* lat) {
  hipLaunchKernelGGL(k_scatter_compact<R>, dim3(grid_for(nfv * d)), dim3(256), 0, st, nfv, d, f2l, c, lat);
}
template <typename R>
void launch_gather_compact(hipStream_t st, int64_t nfv, int d, const int32_t* f2l, const R* lat, R* c) {
  hipLaunchKernelGGL(k_gather_compact<R>, dim3(grid_for(nfv * d)), dim3(256), 0, st, nfv, d, f2l, lat, c);
}
template <typename R>
void launch_minres_w(hipStream_t st, int64_t n, const R* v, R* w1, const R* w2, R* x, double a, double b, double c,
                     double phi) {
  hipLaunchKernelGGL(k_minres_w<R>, dim3(grid_for(n)), dim3(256), 0, st, n, v, w1, w2, x, a, b, c, phi);
}
template <typename A, typename B>
void launch_scale_convert(hipStream_t st, int64_t n, double a, const A* x, B* y, int add) {
  hipLaunchKernelGGL((k_scale_convert<A, B>), dim3(grid_for(n)), dim3(256), 0, st, n, a, x, y, add);
}

#define MCS_INST(R)                                                                                             \
  template void launch_elem_apply<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, const R*, R*, R*, int); \
  template void launch_facet_sum<R>(hipStream_t, const SolveParams&, const R*, const R*, R, R*);               \
  template void launch_ext_pre<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, const R*, R*, R*);        \
  template void launch_ext_post<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, const R*, const R*, R*); \
  template void launch_smooth_phase<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, int32_t, int32_t, R*, \
                                       const R*, R*, int, int64_t);                                            \
  template void launch_block_jacobi<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, const R*, R*);      \
  template void launch_smooth_last<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, int32_t, int32_t, R*,   \
                                      const R*, const R*);                                                      \
  template void launch_ycorr<R>(hipStream_t, const SolveParams&, const R*, const int32_t*, const int32_t*,       \
                                const R*, R*);                                                                  \
  template void launch_edt<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, const R*, R*, int64_t,         \
                              const int32_t*, const int32_t*, const int32_t*, R*, int);                        \
  template void launch_ed<R>(hipStream_t, const SolveParams&, const OpPtrs<R>&, const int32_t*, const int32_t*, \
                             const R*, R*, int, int);                                                          \
  template void launch_mg_point<R>(hipStream_t, int, const MGLevelDev&, int);                                  \
  template void launch_mg_restrict<R>(hipStream_t, int, const MGLevelDev&, const MGLevelDev&);                 \
  template void launch_mg_prolong<R>(hipStream_t, int, const MGLevelDev&, const MGLevelDev&);                  \
  template void launch_mg_coarse<R>(hipStream_t, const double*, const int32_t*, int, const MGLevelDev&);       \
  template void launch_elem_press<R>(hipStream_t, const SolveParams&, const R*, const R*, R*, int);            \
  template void launch_axpby<R>(hipStream_t, int64_t, double, const R*, double, R*);                           \
  template void launch_fill<R>(hipStream_t, int64_t, R, R*);                                                   \
  template void launch_dot<R>(hipStream_t, int64_t, const R*, const R*, double*, double*);                  \
  template void launch_minres_w<R>(hipStream_t, int64_t, const R*, R*, const R*, R*, double, double, double, double); \
  template void launch_scatter_compact<R>(hipStream_t, int64_t, int, const int32_t*, const R*, R*);             \
  template void launch_gather_compact<R>(hipStream_t, int64_t, int, const int32_t*, const R*, R*);

MCS_INST(double)
MCS_INST(float)
template void launch_convert<double, float>(hipStream_t, int64_t, const double*, float*);
template void launch_convert<float, double>(hipStream_t, int64_t, const float*, double*);
template void launch_scale_convert<double, float>(hipStream_t, int64_t, double, const double*, float*, int);
template void launch_scale_convert<float, double>(hipStream_t, int64_t, double, const float*, double*, int);
template void launch_scale_convert<double, double>(hipStream_t, int64_t, double, const double*, double*, int);

}  // namespace mcs
