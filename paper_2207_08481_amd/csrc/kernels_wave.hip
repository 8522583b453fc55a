// Element kernels of the lowest-order method (k = 1, Sec. 7 "The lowest order
// case"): no velocity bubbles, facet blocks of 6 dofs (n_d = 24) and one
// pressure dof per element.  The general element kernels give a whole workgroup to an element
// and synchronise it between phases; with 24 rows that leaves most lanes idle
// and the barriers on the critical path.  Here one wave owns one element
// (four per workgroup) and its lanes own the element's rows: no workgroup
// barriers, the facet values are passed between lanes by shuffles.
#include "kernels_common.h"
#include "launch.h"

namespace mcs {

namespace {

template <typename R>
__device__ inline R lane_sum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Row of the element's facet rows -> BDM index (facet function), or -1 for
// the tangential and omega rows.
__device__ inline int facet_row_bdm(const Sizes& s, int row) {
  const int f = row / s.nfb, q = row % s.nfb;
  return q < s.nF ? f * s.nF + q : -1;
}

// Lane t < n_d: the element's facet value x_d[t] (Dirichlet facets: the lift,
// else 0).
template <typename R>
__device__ inline R gather_lane(const SolveParams& P, const R* __restrict__ x, int64_t e, int lane) {
  const Sizes& s = P.s;
  if (lane >= s.nd) return R(0);
  const int f = lane / s.nfb, q = lane % s.nfb;
  const int g = P.elem_ff[e * (s.d + 1) + f];
  return g >= 0 ? x[P.off_f + (int64_t)g * s.nfb + q] : (P.xD ? (R)P.xD[e * s.nd + lane] : R(0));
}

constexpr int EPB = 4;   // elements (waves) per workgroup

}  // namespace

// The contract of k_elem_apply for n_b = 0 and n_p = 1: flags 1 = A^d x_d,
// 2 = + B^T p, 4 = p <- B u, 8 = A^d only, 16 = zero pressure rows when B u
// is not requested.  Facet rows go to escr[e][n_d] (summed per facet by
// k_facet_sum), the pressure row to y.  B_T[q][row] = -|det J| / det J
// Bp^[q][iu(row)] for the facet functions.  Four elements per wave, 16 lanes
// each; a lane owns two adjacent rows (n_d <= 32, even) and loads both of
// their entries of a column of A^d at once (A^d symmetric: column = row).
template <typename R, typename MA>
__global__ void __launch_bounds__(256) k_elem_apply_wave(SolveParams P, MA MAd, const R* __restrict__ x,
                                                         R* __restrict__ y, R* __restrict__ escr, int flags) {
  typedef R r2v __attribute__((ext_vector_type(2)));
  constexpr int LPE = 16;                               // lanes per element
  const Sizes s = P.s;
  const int nd = s.nd;
  const int lane = threadIdx.x & 63, sub = lane & (LPE - 1), es = lane / LPE;
  const int gbase = lane - sub;                         // first lane of the element's group
  const bool doA = flags & 1, doBT = flags & 2, doBu = flags & 4;
  const int r0 = 2 * sub;                               // the lane's rows r0, r0 + 1
  const bool act = r0 < nd;
  const int rc = act ? r0 : nd - 2;                     // inactive lanes read valid rows
  const int iu0 = act ? facet_row_bdm(s, r0) : -1, iu1 = act ? facet_row_bdm(s, r0 + 1) : -1;
  const double bp0 = iu0 >= 0 ? P.rBp[iu0] : 0.0, bp1 = iu1 >= 0 ? P.rBp[iu1] : 0.0;
  const int64_t per = (int64_t)(blockDim.x / 64) * 4;   // elements per workgroup
  for (int64_t e0 = (int64_t)blockIdx.x * per + (threadIdx.x >> 6) * 4; e0 < P.ne; e0 += (int64_t)gridDim.x * per) {
    // every lane takes part in the shuffles; slots past the end or switched
    // off read a valid element and store nothing
    const int64_t eslot = e0 + es;
    const bool live = eslot < P.ne && !elem_off(P, eslot);
    const int64_t e = eslot < P.ne ? eslot : P.ne - 1;
    R xd0 = R(0), xd1 = R(0);
    if ((doA || doBu) && act) {
      xd0 = gather_lane(P, x, e, r0);
      xd1 = gather_lane(P, x, e, r0 + 1);
    }
    const double sf = P.detJ[e] > 0 ? -1.0 : 1.0;
    R acc0 = R(0), acc1 = R(0);
    if (doA) {
      const size_t a0 = (size_t)e * nd * nd + rc;
#pragma unroll 8
      for (int j = 0; j < nd; ++j) {
        const R xj = (j & 1) ? __shfl(xd1, gbase + (j >> 1), 64) : __shfl(xd0, gbase + (j >> 1), 64);
        R m0, m1;
        if constexpr (std::is_same<MA, MatP<R>>::value) {
          const r2v m = *reinterpret_cast<const r2v*>(MAd.p + a0 + (size_t)j * nd);
          m0 = m.x;
          m1 = m.y;
        } else {
          m0 = MAd(a0 + (size_t)j * nd);
          m1 = MAd(a0 + (size_t)j * nd + 1);
        }
        acc0 += m0 * xj;
        acc1 += m1 * xj;
      }
    }
    if (doBT) {
      const double pe = (double)x[P.off_p + e];
      if (iu0 >= 0) acc0 += (R)(sf * (bp0 * pe));
      if (iu1 >= 0) acc1 += (R)(sf * (bp1 * pe));
    }
    if (live && act) {
      r2v o;
      o.x = acc0;
      o.y = acc1;
      *reinterpret_cast<r2v*>(escr + e * nd + r0) = o;
    }
    if (doBu) {
      double a = (iu0 >= 0 ? bp0 * (sf * (double)xd0) : 0.0) + (iu1 >= 0 ? bp1 * (sf * (double)xd1) : 0.0);
#pragma unroll
      for (int off = LPE / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
      if (live && sub == 0) y[P.off_p + e] = (R)a;
    } else if (!(flags & 8) && (flags & 16) && live && sub == 0) {
      y[P.off_p + e] = R(0);
    }
  }
}

// The contract of k_elem_press for n_b = 0 and n_p = 1:
// y_p = (nu_T / |det J|) Mp^-1_ref (r_p - B a) (with_B = 0: without B a).
template <typename R>
__global__ void __launch_bounds__(256) k_elem_press_wave(SolveParams P, const R* __restrict__ a,
                                                         const R* __restrict__ r, R* __restrict__ y, int with_B) {
  const Sizes s = P.s;
  const int lane = threadIdx.x & 63;
  const int iu = lane < s.nd ? facet_row_bdm(s, lane) : -1;
  const double bp = iu >= 0 ? P.rBp[iu] : 0.0;
  const double mpi = P.rMpinv[0];
  for (int64_t e = (int64_t)blockIdx.x * EPB + (threadIdx.x >> 6); e < P.ne; e += (int64_t)gridDim.x * EPB) {
    if (elem_off(P, e)) continue;
    const double det = P.detJ[e];
    double ba = 0.0;
    if (with_B) {
      const double sf = det > 0 ? -1.0 : 1.0;
      const R ad = gather_lane(P, a, e, lane);
      ba = lane_sum(iu >= 0 ? bp * (sf * (double)ad) : 0.0);
    }
    if (lane == 0) y[P.off_p + e] = (R)(P.nu[e] / fabs(det) * (mpi * ((double)r[P.off_p + e] - ba)));
  }
}

static unsigned wave_grid(int64_t ne) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((ne + EPB - 1) / EPB, 1 << 20));
}

template <typename R>
void launch_elem_apply_wave(hipStream_t st, const SolveParams& P, const OpPtrs<R>& O, const R* x, R* y, R* escr,
                            int flags) {
  if (P.s.nd > 32 || P.s.nd % 2) {   // the kernel's lane layout: two rows per lane, 16 lanes
    launch_elem_apply<R>(st, P, O, x, y, escr, flags);
    return;
  }
  // four elements per wave
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((P.ne + 4 * EPB - 1) / (4 * EPB), 1 << 20))),
      b(64 * EPB);
  if constexpr (sizeof(R) == 8) {
    if (!O.Ad) {   // split storage: FP64 entries as FP32 hi + lo
      hipLaunchKernelGGL((k_elem_apply_wave<R, MatHL>), g, b, 0, st, P, MatHL{O.hAd, O.lAd}, x, y, escr, flags);
      return;
    }
  }
  hipLaunchKernelGGL((k_elem_apply_wave<R, MatP<R>>), g, b, 0, st, P, MatP<R>{O.Ad}, x, y, escr, flags);
}
template <typename R>
void launch_elem_press_wave(hipStream_t st, const SolveParams& P, const R* a, const R* r, R* y, int with_B) {
  hipLaunchKernelGGL(k_elem_press_wave<R>, dim3(wave_grid(P.ne)), dim3(64 * EPB), 0, st, P, a, r, y, with_B);
}

template void launch_elem_apply_wave<double>(hipStream_t, const SolveParams&, const OpPtrs<double>&, const double*,
                                             double*, double*, int);
template void launch_elem_apply_wave<float>(hipStream_t, const SolveParams&, const OpPtrs<float>&, const float*,
                                            float*, float*, int);
template void launch_elem_press_wave<double>(hipStream_t, const SolveParams&, const double*, const double*, double*,
                                             int);
template void launch_elem_press_wave<float>(hipStream_t, const SolveParams&, const float*, const float*, float*, int);

}  // namespace mcs
