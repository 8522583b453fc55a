// Batched preconditioned MINRES over a union of member problems: per-member
// inner products, Lanczos updates, Givens recurrences (Paige-Saunders) and
// iterate updates with the scalars resident in device memory, so that a run
// of iterations needs no host round trip and can be captured in a graph.
// Every kernel skips the tiles of members whose mask entry is zero.
#include <cmath>

#include "kernels_common.h"
#include "launch.h"

namespace mcs {

namespace {

__device__ inline double bwave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline bool tile_on(const SegDev& S, const SegTile& t) { return S.active[t.prob] != 0; }

// partial[t] = sum over tile t of a_i b_i (FP64 accumulation)
template <typename R>
__global__ void __launch_bounds__(256) k_seg_dot(SegDev S, const R* __restrict__ a, const R* __restrict__ b) {
  __shared__ double sh[4];
  for (int64_t ti = blockIdx.x; ti < S.ntiles; ti += gridDim.x) {
    const SegTile t = S.tiles[ti];
    if (!tile_on(S, t)) continue;
    double acc = 0.0;
    for (int i = threadIdx.x; i < t.len; i += blockDim.x) acc += (double)a[t.start + i] * (double)b[t.start + i];
    acc = bwave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) S.partial[ti] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
  }
}

// st[field][p] = sum of the member's tile partials (one wave per member)
__global__ void k_seg_reduce(SegDev S, int field) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= S.nprob || !S.active[p]) return;
  double acc = 0.0;
  for (int t = S.tile_off[p] + lane; t < S.tile_off[p + 1]; t += 64) acc += S.partial[t];
  acc = bwave_sum(acc);
  if (lane == 0) S.st[field * S.nprob + p] = acc;
}

// dst = src * st[field] (or / st[field] when inv)
template <typename R>
__global__ void k_seg_scale(SegDev S, const R* __restrict__ src, R* __restrict__ dst, int field, int inv) {
  for (int64_t ti = blockIdx.x; ti < S.ntiles; ti += gridDim.x) {
    const SegTile t = S.tiles[ti];
    if (!tile_on(S, t)) continue;
    const double f = S.st[field * S.nprob + t.prob];
    const double c = inv ? 1.0 / f : f;
    for (int i = threadIdx.x; i < t.len; i += blockDim.x) dst[t.start + i] = (R)(c * (double)src[t.start + i]);
  }
}

// y -= (st[num] / st[den]) x, only for members with its > min_its
template <typename R>
__global__ void k_seg_axpy_ratio(SegDev S, const R* __restrict__ x, R* __restrict__ y, int num, int den, int min_its) {
  for (int64_t ti = blockIdx.x; ti < S.ntiles; ti += gridDim.x) {
    const SegTile t = S.tiles[ti];
    if (!tile_on(S, t) || S.its[t.prob] < min_its) continue;
    const double c = S.st[num * S.nprob + t.prob] / S.st[den * S.nprob + t.prob];
    for (int i = threadIdx.x; i < t.len; i += blockDim.x)
      y[t.start + i] = (R)((double)y[t.start + i] - c * (double)x[t.start + i]);
  }
}

// w1 <- cw0 v + cw1 w1 + cw2 w2;  x += phi w1
template <typename R>
__global__ void k_seg_w(SegDev S, const R* __restrict__ v, R* __restrict__ w1, const R* __restrict__ w2,
                        R* __restrict__ x) {
  for (int64_t ti = blockIdx.x; ti < S.ntiles; ti += gridDim.x) {
    const SegTile t = S.tiles[ti];
    if (!tile_on(S, t)) continue;
    const int n = S.nprob, p = t.prob;
    const double a = S.st[ST_CW0 * n + p], b = S.st[ST_CW1 * n + p], c = S.st[ST_CW2 * n + p],
                 phi = S.st[ST_PHI * n + p];
    for (int i = threadIdx.x; i < t.len; i += blockDim.x) {
      const int64_t j = t.start + i;
      const double wn = a * (double)v[j] + b * (double)w1[j] + c * (double)w2[j];
      w1[j] = (R)wn;
      x[j] = (R)((double)x[j] + phi * wn);
    }
  }
}

// y (B) = st[field] * x (A), or y += st[field] * x when add (FP32 <-> FP64)
template <typename A, typename B>
__global__ void k_seg_scale_convert(SegDev S, const A* __restrict__ x, B* __restrict__ y, int field, int inv, int add) {
  for (int64_t ti = blockIdx.x; ti < S.ntiles; ti += gridDim.x) {
    const SegTile t = S.tiles[ti];
    if (!tile_on(S, t)) continue;
    const double f = S.st[field * S.nprob + t.prob];
    const double c = inv ? 1.0 / f : f;
    for (int i = threadIdx.x; i < t.len; i += blockDim.x) {
      const int64_t j = t.start + i;
      const double v = c * (double)x[j];
      y[j] = add ? (B)((double)y[j] + v) : (B)v;
    }
  }
}

// y = a - b on the active tiles (FP64 outer residual)
__global__ void k_seg_sub(SegDev S, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  for (int64_t ti = blockIdx.x; ti < S.ntiles; ti += gridDim.x) {
    const SegTile t = S.tiles[ti];
    if (!tile_on(S, t)) continue;
    for (int i = threadIdx.x; i < t.len; i += blockDim.x) y[t.start + i] = a[t.start + i] - b[t.start + i];
  }
}

// MINRES start: beta1 = sqrt(<r, K-hat^{-1} r>) from st[BB]; a member enters
// the iteration unless beta1 is zero or already below its st[SB1].
__global__ void k_mr_init(SegDev S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S.nprob || !S.active[p]) return;
  const int n = S.nprob;
  double* st = S.st;
  const double b2 = st[ST_BB * n + p];
  S.its[p] = 0;
  S.done[p] = 0;
  st[ST_REL * n + p] = 0.0;
  st[ST_BETA1 * n + p] = 0.0;
  if (!isfinite(b2)) {
    S.status[p] = MCS_ERR_NONFINITE;
    S.active[p] = 0;
    return;
  }
  if (b2 < 0.0) {
    S.status[p] = MCS_ERR_BREAKDOWN;
    S.active[p] = 0;
    return;
  }
  const double beta1 = sqrt(b2);
  st[ST_BETA1 * n + p] = beta1;
  S.status[p] = MCS_OK;
  if (beta1 == 0.0 || beta1 <= st[ST_SB1 * n + p]) {
    S.active[p] = 0;
    return;
  }
  st[ST_BETA * n + p] = beta1;
  st[ST_OLDB * n + p] = 0.0;
  st[ST_DBAR * n + p] = 0.0;
  st[ST_EPS * n + p] = 0.0;
  st[ST_PHIBAR * n + p] = beta1;
  st[ST_CS * n + p] = -1.0;
  st[ST_SN * n + p] = 0.0;
  st[ST_STOP * n + p] = fmax(st[ST_TOL * n + p] * beta1, st[ST_ABS * n + p]);
}

// One Givens step after beta_{k+1} = sqrt(st[BB]): coefficients of the
// direction update, phi, the new residual estimate phibar and the stopping
// decision (applied by k_mr_retire after the iterate update).
__global__ void k_mr_update(SegDev S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S.nprob || !S.active[p]) return;
  const int n = S.nprob;
  double* st = S.st;
  const double alpha = st[ST_ALPHA * n + p], bb = st[ST_BB * n + p];
  if (!isfinite(bb) || !isfinite(alpha)) {
    S.status[p] = MCS_ERR_NONFINITE;
    S.active[p] = 0;
    return;
  }
  if (bb < 0.0) {
    S.status[p] = MCS_ERR_BREAKDOWN;
    S.active[p] = 0;
    return;
  }
  const double cs = st[ST_CS * n + p], sn = st[ST_SN * n + p], dbar = st[ST_DBAR * n + p];
  const double oldeps = st[ST_EPS * n + p], phibar = st[ST_PHIBAR * n + p];
  const double beta = sqrt(bb);
  st[ST_OLDB * n + p] = st[ST_BETA * n + p];
  st[ST_BETA * n + p] = beta;
  const double delta = cs * dbar + sn * alpha;
  const double gbar = sn * dbar - cs * alpha;
  st[ST_EPS * n + p] = sn * beta;
  st[ST_DBAR * n + p] = -cs * beta;
  double gamma = hypot(gbar, beta);
  if (gamma == 0.0) gamma = 1e-300;
  const double cs2 = gbar / gamma, sn2 = beta / gamma;
  st[ST_CS * n + p] = cs2;
  st[ST_SN * n + p] = sn2;
  st[ST_PHI * n + p] = cs2 * phibar;
  const double pb = sn2 * phibar;
  st[ST_PHIBAR * n + p] = pb;
  st[ST_CW0 * n + p] = 1.0 / gamma;
  st[ST_CW1 * n + p] = -oldeps / gamma;
  st[ST_CW2 * n + p] = -delta / gamma;
  const int it = S.its[p] + 1;
  S.its[p] = it;
  st[ST_REL * n + p] = pb / st[ST_BETA1 * n + p];
  if (pb <= st[ST_STOP * n + p]) {
    S.done[p] = 1;
  } else if (it >= S.maxit) {
    S.done[p] = 1;
    S.status[p] = MCS_ERR_NOT_CONVERGED;
  }
}

__global__ void k_mr_retire(SegDev S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S.nprob) return;
  if (S.done[p]) S.active[p] = 0;
}

// Mean-zero pressure per member (one workgroup per member):
// x_p -= (int p / |Omega|) * (coefficients of p = 1).
__global__ void __launch_bounds__(256) k_batch_pmean(SolveParams P, const int64_t* __restrict__ pe0,
                                                     const double* __restrict__ pmom, const double* __restrict__ pconst,
                                                     double* __restrict__ x) {
  __shared__ double sh[2][256];
  const int np = P.s.np;
  const double fd = P.s.d == 2 ? 2.0 : 6.0;
  const int64_t e0 = pe0[blockIdx.x], e1 = pe0[blockIdx.x + 1];
  double a = 0.0, v = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double vol = fabs(P.detJ[e]) / fd;
    double t = 0.0;
    for (int q = 0; q < np; ++q) t += pmom[q] * x[P.off_p + e * np + q];
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
  const double m = sh[0][0] / sh[1][0];
  for (int64_t i = e0 * np + threadIdx.x; i < e1 * np; i += 256) x[P.off_p + i] -= m * pconst[i % np];
}

static unsigned tgrid(const SegDev& S) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(S.ntiles, 1 << 20)); }
static unsigned pgrid(int n, int per) { return (unsigned)std::max(1, (n + per - 1) / per); }

}  // namespace

template <typename R>
void launch_seg_dot(hipStream_t st, const SegDev& S, const R* a, const R* b, int field) {
  hipLaunchKernelGGL(k_seg_dot<R>, dim3(tgrid(S)), dim3(256), 0, st, S, a, b);
  hipLaunchKernelGGL(k_seg_reduce, dim3(pgrid(S.nprob, 4)), dim3(256), 0, st, S, field);
}
template <typename R>
void launch_seg_scale(hipStream_t st, const SegDev& S, const R* src, R* dst, int field, int inv) {
  hipLaunchKernelGGL(k_seg_scale<R>, dim3(tgrid(S)), dim3(256), 0, st, S, src, dst, field, inv);
}
template <typename R>
void launch_seg_axpy_ratio(hipStream_t st, const SegDev& S, const R* x, R* y, int num, int den, int min_its) {
  hipLaunchKernelGGL(k_seg_axpy_ratio<R>, dim3(tgrid(S)), dim3(256), 0, st, S, x, y, num, den, min_its);
}
template <typename R>
void launch_seg_w(hipStream_t st, const SegDev& S, const R* v, R* w1, const R* w2, R* x) {
  hipLaunchKernelGGL(k_seg_w<R>, dim3(tgrid(S)), dim3(256), 0, st, S, v, w1, w2, x);
}
template <typename A, typename B>
void launch_seg_scale_convert(hipStream_t st, const SegDev& S, const A* x, B* y, int field, int inv, int add) {
  hipLaunchKernelGGL((k_seg_scale_convert<A, B>), dim3(tgrid(S)), dim3(256), 0, st, S, x, y, field, inv, add);
}
void launch_seg_sub(hipStream_t st, const SegDev& S, const double* a, const double* b, double* y) {
  hipLaunchKernelGGL(k_seg_sub, dim3(tgrid(S)), dim3(256), 0, st, S, a, b, y);
}
void launch_mr_init(hipStream_t st, const SegDev& S) {
  hipLaunchKernelGGL(k_mr_init, dim3(pgrid(S.nprob, 256)), dim3(256), 0, st, S);
}
void launch_mr_update(hipStream_t st, const SegDev& S) {
  hipLaunchKernelGGL(k_mr_update, dim3(pgrid(S.nprob, 256)), dim3(256), 0, st, S);
}
void launch_mr_retire(hipStream_t st, const SegDev& S) {
  hipLaunchKernelGGL(k_mr_retire, dim3(pgrid(S.nprob, 256)), dim3(256), 0, st, S);
}
void launch_batch_pmean(hipStream_t st, const SolveParams& P, int nprob, const int64_t* pe0, const double* pmom,
                        const double* pconst, double* x) {
  hipLaunchKernelGGL(k_batch_pmean, dim3(nprob), dim3(256), 0, st, P, pe0, pmom, pconst, x);
}

#define MCS_BINST(R)                                                                                   \
  template void launch_seg_dot<R>(hipStream_t, const SegDev&, const R*, const R*, int);                 \
  template void launch_seg_scale<R>(hipStream_t, const SegDev&, const R*, R*, int, int);                \
  template void launch_seg_axpy_ratio<R>(hipStream_t, const SegDev&, const R*, R*, int, int, int);      \
  template void launch_seg_w<R>(hipStream_t, const SegDev&, const R*, R*, const R*, R*);
MCS_BINST(double)
MCS_BINST(float)
template void launch_seg_scale_convert<double, float>(hipStream_t, const SegDev&, const double*, float*, int, int, int);
template void launch_seg_scale_convert<float, double>(hipStream_t, const SegDev&, const float*, double*, int, int, int);

}  // namespace mcs
