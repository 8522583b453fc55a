// Reference-element tables for the MCS element kernels (host, computed once
// per dimension and order).  Integrals use collapsed (Duffy) Gauss-Legendre
// rules on the reference simplex and its facets, exact for the polynomial
// degrees involved (<= 2k+1).
//
// Spaces (Sec. 3 of the paper): BDM^k velocity split into normal bubbles and
// facet functions (Sec. 4.2, "Static condensation of high order velocity
// functions"), hat V_h facet tangential fields, P^{k-1} pressure, trace-free
// stress polynomials P^k(T, D) described by an orthonormal scalar basis, and
// the top-degree facet polynomials that define the nt-trace constraint of
// Sigma_h (eq. fes_Sigma).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <numeric>
#include <stdexcept>

#include "mcs_internal.h"

namespace mcs {

namespace {

using MI = std::vector<int>;

void multi_rec(int nvars, int degree, MI& cur, std::vector<MI>& out) {
  if (nvars == 1) {
    cur.push_back(degree);
    out.push_back(cur);
    cur.pop_back();
    return;
  }
  for (int a = degree; a >= 0; --a) {
    cur.push_back(a);
    multi_rec(nvars - 1, degree - a, cur, out);
    cur.pop_back();
  }
}

// Multi-indices of N^nvars with |alpha| = degree, lexicographically descending.
std::vector<MI> multi_indices(int nvars, int degree) {
  std::vector<MI> out;
  MI cur;
  multi_rec(nvars, degree, cur, out);
  return out;
}

int64_t binom(int n, int r) {
  if (r < 0 || r > n) return 0;
  int64_t v = 1;
  for (int i = 1; i <= r; ++i) v = v * (n - r + i) / i;
  return v;
}

double fact(int n) {
  double v = 1;
  for (int i = 2; i <= n; ++i) v *= i;
  return v;
}

// Solves M x = b (n x n, row-major, overwritten) by Gaussian elimination with
// partial pivoting; b receives x.
void solve_dense(std::vector<double>& M, int n, std::vector<double>& b) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)p * n + c])) p = r;
    if (p != c) {
      for (int t = 0; t < n; ++t) std::swap(M[(size_t)c * n + t], M[(size_t)p * n + t]);
      std::swap(b[c], b[p]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = M[(size_t)r * n + c] / M[(size_t)c * n + c];
      if (f == 0.0) continue;
      for (int t = c; t < n; ++t) M[(size_t)r * n + t] -= f * M[(size_t)c * n + t];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double t = b[c];
    for (int j = c + 1; j < n; ++j) t -= M[(size_t)c * n + j] * b[j];
    b[c] = t / M[(size_t)c * n + c];
  }
}

// (1/|F|) int_F mu^a mu^b over a simplex with nvar barycentric coordinates
// (exact: (nvar-1)! (a+b)! / (|a|+|b|+nvar-1)!)
double simplex_moment2(const MI& a, const MI& b) {
  const int nvar = (int)a.size();
  int tot = 0;
  double num = fact(nvar - 1);
  for (int j = 0; j < nvar; ++j) {
    num *= fact(a[j] + b[j]);
    tot += a[j] + b[j];
  }
  return num / fact(tot + nvar - 1);
}

// Gauss-Legendre nodes/weights on [0, 1] (Newton iteration on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pnm1 = (n == 1) ? 1.0 : p0;
      double dp = n * (z * pn - pnm1) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1;
    double pnm1 = (n == 1) ? 1.0 : p0;
    double dp = n * (z * pn - pnm1) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2) P'^2) scaled by 1/2
  }
}

struct Rule {
  std::vector<std::vector<double>> lam;  // barycentric coordinates (dim+1)
  std::vector<double> w;                 // weights, sum = 1/dim!
};

// Collapsed rule on the reference dim-simplex, n points per direction.
Rule simplex_rule(int dim, int n) {
  std::vector<double> g, gw;
  gauss_legendre01(n, g, gw);
  Rule R;
  if (dim == 1) {
    for (int i = 0; i < n; ++i) {
      R.lam.push_back({1.0 - g[i], g[i]});
      R.w.push_back(gw[i]);
    }
  } else if (dim == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double x = g[i], y = g[j] * (1.0 - g[i]);
        R.lam.push_back({1.0 - x - y, x, y});
        R.w.push_back(gw[i] * gw[j] * (1.0 - g[i]));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l) {
          double x = g[i], y = g[j] * (1.0 - g[i]), z = g[l] * (1.0 - g[i]) * (1.0 - g[j]);
          R.lam.push_back({1.0 - x - y - z, x, y, z});
          R.w.push_back(gw[i] * gw[j] * gw[l] * (1.0 - g[i]) * (1.0 - g[i]) * (1.0 - g[j]));
        }
  }
  return R;
}

double mono(const std::vector<double>& lam, const MI& a) {
  double v = 1.0;
  for (size_t j = 0; j < a.size(); ++j)
    for (int p = 0; p < a[j]; ++p) v *= lam[j];
  return v;
}

// d/dxhat_s of lambda^alpha on the reference simplex (lambda_0 = 1 - sum x).
void mono_grad(const std::vector<double>& lam, const MI& a, int d, double* g) {
  for (int s = 0; s < d; ++s) g[s] = 0.0;
  for (int j = 0; j <= d; ++j) {
    if (a[j] == 0) continue;
    MI b = a;
    b[j] -= 1;
    double v = a[j] * mono(lam, b);
    if (j == 0)
      for (int s = 0; s < d; ++s) g[s] -= v;
    else
      g[j - 1] += v;
  }
}

std::vector<double> dense_inverse(std::vector<double> A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) throw std::runtime_error("singular reference matrix");
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(A[c * n + j], A[piv * n + j]);
        std::swap(I[c * n + j], I[piv * n + j]);
      }
    double inv = 1.0 / A[c * n + c];
    for (int j = 0; j < n; ++j) {
      A[c * n + j] *= inv;
      I[c * n + j] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[r * n + j] -= f * A[c * n + j];
        I[r * n + j] -= f * I[c * n + j];
      }
    }
  }
  return I;
}

// Orthonormal, degree-graded basis of P^k on the reference nvar-simplex
// w.r.t. (1/|T|) int, as coefficients over the degree-k Bernstein polynomials
// B_beta = k!/beta! lambda^beta (beta over nvar+1 barycentric components):
// psi_a = sum_beta C[a][beta] B_beta.  Built degree by degree: the Bernstein
// polynomials of degree j = 0..k (raised to degree k) are orthonormalised
// against all earlier functions by Gram-Schmidt, twice, in extended precision
// with the exact Gram matrix; the functions that add nothing (already in the
// span of lower degrees) are dropped.  So psi_0 .. psi_{dim P^{k-1} - 1} span
// P^{k-1} and the rest is its orthogonal complement in P^k.  (A Cholesky
// factor of the monomial Gram matrix would lose orthogonality: its condition
// number is ~5e10 at k = 5 in 3D.)
struct PolyBasis {
  int nvar = 0, k = 0, n = 0;
  std::vector<MI> bern;          // degree-k multi-indices (nvar+1 components)
  std::vector<long double> C;    // [n][n]
  std::vector<long double> bfac; // k!/beta!
  // values of all psi_a at barycentric point lam (nvar+1 components)
  void eval(const std::vector<double>& lam, double* out) const {
    std::vector<long double> b(n);
    for (int j = 0; j < n; ++j) {
      long double v = bfac[j];
      for (int t = 0; t <= nvar; ++t)
        for (int p = 0; p < bern[j][t]; ++p) v *= (long double)lam[t];
      b[j] = v;
    }
    for (int a = 0; a < n; ++a) {
      long double t = 0;
      for (int j = 0; j < n; ++j) t += C[(size_t)a * n + j] * b[j];
      out[a] = (double)t;
    }
  }
};

long double lfact(int n) {
  long double v = 1;
  for (int i = 2; i <= n; ++i) v *= i;
  return v;
}

PolyBasis orthonormal_basis(int nvar, int k) {
  PolyBasis P;
  P.nvar = nvar;
  P.k = k;
  P.bern = multi_indices(nvar + 1, k);
  const int n = (int)P.bern.size();
  P.n = n;
  std::map<MI, int> idx;
  for (int j = 0; j < n; ++j) idx[P.bern[j]] = j;
  P.bfac.resize(n);
  for (int j = 0; j < n; ++j) {
    long double den = 1;
    for (int t = 0; t <= nvar; ++t) den *= lfact(P.bern[j][t]);
    P.bfac[j] = lfact(k) / den;
  }
  // exact Gram matrix: (1/|T|) int B_a B_b = (k!)^2/(a! b!) (a+b)! nvar! / (2k+nvar)!
  std::vector<long double> G((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double v = P.bfac[i] * P.bfac[j] * lfact(nvar) / lfact(2 * k + nvar);
      for (int t = 0; t <= nvar; ++t) v *= lfact(P.bern[i][t] + P.bern[j][t]);
      G[(size_t)i * n + j] = v;
    }
  auto dot = [&](const std::vector<long double>& x, const std::vector<long double>& y) {
    long double s = 0;
    for (int i = 0; i < n; ++i) {
      long double t = 0;
      for (int j = 0; j < n; ++j) t += G[(size_t)i * n + j] * y[j];
      s += x[i] * t;
    }
    return s;
  };
  std::vector<std::vector<long double>> Q;
  for (int deg = 0; deg <= k; ++deg) {
    for (auto& g : multi_indices(nvar + 1, deg)) {
      // B^deg_g raised to degree k: sum over h (|h| = k - deg) of
      // (deg!/g!) ((k-deg)!/h!) / (k!/(g+h)!) B^k_{g+h}
      std::vector<long double> v(n, 0.0L);
      long double cg = lfact(deg);
      for (int t = 0; t <= nvar; ++t) cg /= lfact(g[t]);
      for (auto& h : multi_indices(nvar + 1, k - deg)) {
        MI gh(nvar + 1);
        long double ch = lfact(k - deg);
        for (int t = 0; t <= nvar; ++t) {
          gh[t] = g[t] + h[t];
          ch /= lfact(h[t]);
        }
        const int j = idx[gh];
        v[j] += cg * ch / P.bfac[j];
      }
      const long double n0 = std::sqrt(dot(v, v));
      for (int pass = 0; pass < 2; ++pass)
        for (auto& q : Q) {
          const long double c = dot(q, v);
          for (int i = 0; i < n; ++i) v[i] -= c * q[i];
        }
      const long double nv = std::sqrt(dot(v, v));
      if (nv < 1e-9L * n0) continue;   // in the span of the lower degrees
      for (int i = 0; i < n; ++i) v[i] /= nv;
      Q.push_back(v);
    }
  }
  if ((int)Q.size() != n) throw std::runtime_error("orthonormal basis: wrong dimension");
  P.C.resize((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int j = 0; j < n; ++j) P.C[(size_t)a * n + j] = Q[a][j];
  return P;
}

}  // namespace

Sizes make_sizes(int d, int k) {
  Sizes s{};
  s.d = d;
  s.k = k;
  s.m = k + 1;
  s.nv = d + 1;
  s.ns = (int)binom(k + d, d);
  s.nsm1 = (int)binom(k - 1 + d, d);
  s.nFk = (int)binom(k + d - 1, d - 1);
  s.nFkm1 = (int)binom(k - 1 + d - 1, d - 1);
  s.nu = d * s.ns;
  s.nF = s.nFk;
  s.nb = s.nu - (d + 1) * s.nF;
  s.nh = (d - 1) * s.nFkm1;
  s.nw = k == 1 ? 1 : 0;
  s.nfb = s.nF + s.nh + s.nw;
  s.nd = (d + 1) * s.nfb;
  s.nA = s.nu + (d + 1) * (s.nh + s.nw);
  s.np = s.nsm1;
  s.nsym = d * (d + 1) / 2 - 1;
  s.nskew = d * (d - 1) / 2;
  s.sklo = k == 1 ? 0 : s.nsm1;
  s.nsig = s.nsym * s.ns + s.nskew * (s.ns - s.sklo);
  s.nlam = (d + 1) * (d - 1) * (s.nFk - s.nFkm1);
  s.nlat = (int)binom(s.m + d, d);
  return s;
}

int perm_index(const int* perm, int nv) {
  // rank among permutations of 0..nv-1 in lexicographic order
  int r = 0;
  for (int i = 0; i < nv; ++i) {
    int smaller = 0;
    for (int j = i + 1; j < nv; ++j)
      if (perm[j] < perm[i]) ++smaller;
    r = r * (nv - i) + smaller;
  }
  return r;
}

RefTables build_ref_tables(int d, int k) {
  RefTables T;
  Sizes s = make_sizes(d, k);
  T.s = s;
  const int nv = s.nv;

  // ---------------- velocity basis description
  struct VFun {
    MI alpha;
    double w[3];  // constant vector (reference), scaled
  };
  std::vector<VFun> phis;
  auto evec = [&](int j, double* out) {  // reference vertex coordinates
    for (int r = 0; r < d; ++r) out[r] = (j > 0 && r == j - 1) ? 1.0 : 0.0;
  };
  for (auto& a : multi_indices(nv, k)) {
    std::vector<int> S;
    for (int j = 0; j < nv; ++j)
      if (a[j] > 0) S.push_back(j);
    if (S.size() < 2) continue;
    for (size_t t = 1; t < S.size(); ++t) {
      VFun f;
      f.alpha = a;
      double ea[3], e0[3];
      evec(S[t], ea);
      evec(S[0], e0);
      for (int r = 0; r < 3; ++r) f.w[r] = r < d ? ea[r] - e0[r] : 0.0;
      phis.push_back(f);
    }
  }
  if ((int)phis.size() != s.nb) throw std::runtime_error("bubble count mismatch");
  for (int f = 0; f < nv; ++f) {
    std::vector<int> fv;
    for (int j = 0; j < nv; ++j)
      if (j != f) fv.push_back(j);
    double sign = (f % 2 == 0) ? 1.0 : -1.0;
    for (auto& beta : multi_indices(d, k)) {
      VFun F;
      F.alpha.assign(nv, 0);
      for (int j = 0; j < d; ++j) F.alpha[fv[j]] = beta[j];
      int j0 = -1;
      for (int j = 0; j < d; ++j)
        if (beta[j] > 0) {
          j0 = fv[j];
          break;
        }
      double ej[3], ef[3];
      evec(j0, ej);
      evec(f, ef);
      for (int r = 0; r < 3; ++r) F.w[r] = r < d ? sign * fact(d - 1) * (ej[r] - ef[r]) : 0.0;
      phis.push_back(F);
    }
  }
  if ((int)phis.size() != s.nu) throw std::runtime_error("BDM count mismatch");

  auto phi_eval = [&](const std::vector<double>& lam, double* val /*[nu][d]*/,
                      double* grad /*[nu][d][d]*/, double* div /*[nu]*/) {
    for (int i = 0; i < s.nu; ++i) {
      double m = mono(lam, phis[i].alpha);
      double g[3];
      mono_grad(lam, phis[i].alpha, d, g);
      double dv = 0;
      for (int r = 0; r < d; ++r) {
        if (val) val[i * d + r] = m * phis[i].w[r];
        for (int c = 0; c < d; ++c)
          if (grad) grad[(i * d + r) * d + c] = phis[i].w[r] * g[c];
        dv += phis[i].w[r] * g[r];
      }
      if (div) div[i] = dv;
    }
  };

  // ---------------- orthonormal psi (volume) and top-degree q (facet)
  const PolyBasis Bpsi = orthonormal_basis(d, k);
  auto psi_eval = [&](const std::vector<double>& lam, double* out) { Bpsi.eval(lam, out); };
  const PolyBasis Bq = orthonormal_basis(d - 1, k);
  const int nq = s.nFk - s.nFkm1;
  auto q_eval = [&](const std::vector<double>& mu, double* out) {  // mu: facet barycentrics (d)
    std::vector<double> all(s.nFk);
    Bq.eval(mu, all.data());
    for (int qq = 0; qq < nq; ++qq) out[qq] = all[s.nFkm1 + qq];
  };

  auto Ip = multi_indices(nv, k - 1);   // pressure
  auto IFg = multi_indices(d, k - 1);   // facet tangential scalar part

  // ---------------- lattice Lagrange basis (sorted order), degree m
  auto Ilat = multi_indices(nv, s.m);
  const int nlat = (int)Ilat.size();
  std::vector<double> Vl(nlat * nlat);
  for (int l = 0; l < nlat; ++l) {
    std::vector<double> lam(nv);
    for (int j = 0; j < nv; ++j) lam[j] = double(Ilat[l][j]) / s.m;
    for (int a = 0; a < nlat; ++a) Vl[l * nlat + a] = mono(lam, Ilat[a]);
  }
  std::vector<double> Vinv = dense_inverse(Vl, nlat);  // [alpha][l]

  // ---------------- volume integrals
  T.V.assign((size_t)s.nu * s.ns * d * d, 0.0);
  T.D.assign((size_t)s.nu * s.nu, 0.0);
  T.Bp.assign((size_t)s.np * s.nu, 0.0);
  T.Mp.assign((size_t)s.np * s.np, 0.0);
  T.Rf.assign((size_t)nlat * s.nu * d, 0.0);
  T.Lam.assign((size_t)s.ns * nv, 0.0);
  {
    Rule R = simplex_rule(d, k + 3);
    std::vector<double> val(s.nu * d), grad(s.nu * d * d), dv(s.nu), ps(s.ns), pp(s.np),
        Ll(nlat);
    for (size_t q = 0; q < R.w.size(); ++q) {
      const auto& lam = R.lam[q];
      double w = R.w[q];
      phi_eval(lam, val.data(), grad.data(), dv.data());
      psi_eval(lam, ps.data());
      for (int g = 0; g < s.np; ++g) pp[g] = mono(lam, Ip[g]);
      for (int l = 0; l < nlat; ++l) {
        double t = 0;
        for (int a = 0; a < nlat; ++a) t += Vinv[a * nlat + l] * mono(lam, Ilat[a]);
        Ll[l] = t;
      }
      for (int i = 0; i < s.nu; ++i) {
        for (int a = 0; a < s.ns; ++a)
          for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c)
              T.V[((size_t(i) * s.ns + a) * d + r) * d + c] += w * ps[a] * grad[(i * d + r) * d + c];
        for (int j = 0; j < s.nu; ++j) T.D[i * s.nu + j] += w * dv[i] * dv[j];
        for (int g = 0; g < s.np; ++g) T.Bp[g * s.nu + i] += w * dv[i] * pp[g];
        for (int l = 0; l < nlat; ++l)
          for (int r = 0; r < d; ++r) T.Rf[(size_t(l) * s.nu + i) * d + r] += w * Ll[l] * val[i * d + r];
      }
      for (int g = 0; g < s.np; ++g)
        for (int h = 0; h < s.np; ++h) T.Mp[g * s.np + h] += w * pp[g] * pp[h];
      for (int a = 0; a < s.ns; ++a)
        for (int j = 0; j < nv; ++j) T.Lam[(size_t)a * nv + j] += w * ps[a] * lam[j];
    }
  }
  T.Mpinv = dense_inverse(T.Mp, s.np);

  // ---------------- facet integrals
  T.Bf.assign((size_t)nv * s.nu * s.ns * d, 0.0);
  T.U.assign((size_t)nv * s.nFkm1 * s.ns, 0.0);
  T.L.assign((size_t)nv * nq * s.ns, 0.0);
  {
    Rule R = simplex_rule(d - 1, k + 3);
    for (int f = 0; f < nv; ++f) {
      std::vector<int> fv;
      for (int j = 0; j < nv; ++j)
        if (j != f) fv.push_back(j);
      double meas = (f == 0) ? std::sqrt(double(d)) / fact(d - 1) : 1.0 / fact(d - 1);
      T.facet_measure[f] = meas;
      std::vector<double> val(s.nu * d), ps(s.ns), qv(nq);
      for (size_t q = 0; q < R.w.size(); ++q) {
        const auto& mu = R.lam[q];
        double w = R.w[q] * fact(d - 1) * meas;
        std::vector<double> lam(nv, 0.0);
        for (int j = 0; j < d; ++j) lam[fv[j]] = mu[j];
        phi_eval(lam, val.data(), nullptr, nullptr);
        psi_eval(lam, ps.data());
        q_eval(mu, qv.data());
        for (int i = 0; i < s.nu; ++i)
          for (int a = 0; a < s.ns; ++a)
            for (int r = 0; r < d; ++r)
              T.Bf[((size_t(f) * s.nu + i) * s.ns + a) * d + r] += w * ps[a] * val[i * d + r];
        for (int g = 0; g < s.nFkm1; ++g) {
          double m = mono(mu, IFg[g]);
          for (int a = 0; a < s.ns; ++a) T.U[(size_t(f) * s.nFkm1 + g) * s.ns + a] += w * ps[a] * m;
        }
        for (int qq = 0; qq < nq; ++qq)
          for (int a = 0; a < s.ns; ++a) T.L[(size_t(f) * nq + qq) * s.ns + a] += w * qv[qq] * ps[a];
      }
    }
  }

  // ---------------- lattice permutation maps
  {
    std::vector<int> perm(nv);
    std::iota(perm.begin(), perm.end(), 0);
    int nperm = (int)fact(nv);
    T.latmap.assign((size_t)nperm * nlat, -1);
    std::map<MI, int> idx;
    for (int l = 0; l < nlat; ++l) idx[Ilat[l]] = l;
    do {
      int r = perm_index(perm.data(), nv);
      for (int l = 0; l < nlat; ++l) {
        MI b(nv);
        for (int j = 0; j < nv; ++j) b[j] = Ilat[l][perm[j]];
        T.latmap[(size_t)r * nlat + l] = idx[b];
      }
    } while (std::next_permutation(perm.begin(), perm.end()));
  }

  // ---------------- embedding coefficients: lambda_v in facet Bernstein
  {
    auto IFk = multi_indices(d, k);
    T.cn.assign((size_t)s.nFk * d, 0.0);
    for (int b = 0; b < s.nFk; ++b)
      for (int v = 0; v < d; ++v) {
        if (IFk[b][v] < 1) continue;
        double den = 1.0;
        for (int j = 0; j < d; ++j) den *= fact(IFk[b][j] - (j == v ? 1 : 0));
        T.cn[b * d + v] = fact(k - 1) / den;
      }
    T.ct.assign((size_t)s.nFkm1 * d, 0.0);
    if (k == 1) {
      // the tangential trace of a P1 field is not in hat V_h = P^0: E takes
      // its facet mean (Sec. 7), 1/d of each facet vertex's value
      for (int v = 0; v < d; ++v) T.ct[v] = 1.0 / d;
    } else {
      for (int g = 0; g < s.nFkm1; ++g)
        for (int v = 0; v < d; ++v) {
          if (IFg[g][v] < 1) continue;
          double den = 1.0;
          for (int j = 0; j < d; ++j) den *= fact(IFg[g][j] - (j == v ? 1 : 0));
          T.ct[g * d + v] = fact(k - 2) / den;
        }
    }
  }
  // basis descriptions for point evaluation
  T.phi.assign((size_t)s.nu * (nv + 3), 0.0);
  for (int i = 0; i < s.nu; ++i) {
    for (int j = 0; j < nv; ++j) T.phi[(size_t)i * (nv + 3) + j] = phis[i].alpha[j];
    for (int r = 0; r < 3; ++r) T.phi[(size_t)i * (nv + 3) + nv + r] = phis[i].w[r];
  }
  // bubble coefficients of lambda_v e_r (the P1 field of vertex v, component
  // r, on the reference element) in the BDM basis: lambda_v = lambda_v
  // (sum_j lambda_j)^(k-1) has the degree-k coefficients (k-1)!/(beta-e_v)!,
  // and the d basis functions lambda^beta w_i of one monomial span R^d
  T.Eo.assign((size_t)nv * d * s.nb, 0.0);
  {
    std::map<MI, std::vector<int>> by_alpha;
    for (int i = 0; i < s.nu; ++i) by_alpha[phis[i].alpha].push_back(i);
    for (auto& beta : multi_indices(nv, k)) {
      const std::vector<int>& ids = by_alpha.at(beta);
      if ((int)ids.size() != d) throw std::runtime_error("BDM monomial multiplicity");
      for (int v = 0; v < nv; ++v) {
        if (beta[v] == 0) continue;
        double cf = fact(k - 1);
        for (int j = 0; j < nv; ++j) cf /= fact(beta[j] - (j == v ? 1 : 0));
        for (int r = 0; r < d; ++r) {
          // solve sum_t c_t w_{ids[t]} = cf e_r (d x d, Gaussian elimination with pivoting)
          double M[3][4];
          for (int a = 0; a < d; ++a) {
            for (int t = 0; t < d; ++t) M[a][t] = phis[ids[t]].w[a];
            M[a][d] = a == r ? cf : 0.0;
          }
          for (int c = 0; c < d; ++c) {
            int p = c;
            for (int a = c + 1; a < d; ++a)
              if (std::fabs(M[a][c]) > std::fabs(M[p][c])) p = a;
            for (int t = 0; t <= d; ++t) std::swap(M[c][t], M[p][t]);
            for (int a = 0; a < d; ++a) {
              if (a == c) continue;
              const double f = M[a][c] / M[c][c];
              for (int t = c; t <= d; ++t) M[a][t] -= f * M[c][t];
            }
          }
          for (int t = 0; t < d; ++t)
            if (ids[t] < s.nb) T.Eo[((size_t)v * d + r) * s.nb + ids[t]] = M[t][d] / M[t][t];
        }
      }
    }
  }
  // psi_a in monomial form over the degree-k barycentric powers (the
  // Bernstein factors k!/beta! folded in), for point values of the stress
  T.psi.assign((size_t)s.ns * s.ns, 0.0);
  T.psib.assign((size_t)s.ns * nv, 0.0);
  for (int a = 0; a < s.ns; ++a)
    for (int j = 0; j < s.ns; ++j) T.psi[(size_t)a * s.ns + j] = (double)(Bpsi.C[(size_t)a * s.ns + j] * Bpsi.bfac[j]);
  for (int j = 0; j < s.ns; ++j)
    for (int t = 0; t < nv; ++t) T.psib[(size_t)j * nv + t] = Bpsi.bern[j][t];
  T.pidx.assign((size_t)s.np * nv, 0.0);
  for (int g = 0; g < s.np; ++g)
    for (int j = 0; j < nv; ++j) T.pidx[(size_t)g * nv + j] = Ip[g][j];
  T.pconst.resize(s.np);
  T.pmom.resize(s.np);
  for (int g = 0; g < s.np; ++g) {
    double den = 1.0;
    for (int j = 0; j < nv; ++j) den *= fact(Ip[g][j]);
    T.pconst[g] = fact(k - 1) / den;
    T.pmom[g] = fact(d) * den / fact(k - 1 + d);
  }
  return T;
}

// Dirichlet dofs of every Dirichlet facet from g given on the element
// lattices (degree m, caller vertex order), per element in the local facet
// order of the element ([n_e][n_d]): the normal dofs c with
// sum_beta c_beta mu^beta / |F| the L2 projection of g.n_F onto P^k(F), and
// the tangential dofs the L2 projection of g_t onto V-hat(F) (basis
// mu^gamma t_b, t_b = x_{f_b} - x_{f_0}); for k = 1 also the flux of curl g
// through the facet (omega's dof).  g is interpolated on the facet from the
// lattice points that lie on it.
void dirichlet_lift(const mcs_problem* pb, const double* g_lattice, std::vector<double>& xD) {
  const Sizes& s = pb->sz;
  const int d = pb->d, nv = d + 1, k = s.k, m = s.m;
  const std::vector<MI> Ilat = multi_indices(nv, m);
  const int nlat = (int)Ilat.size();
  const std::vector<MI> Fm = multi_indices(d, m), Fk = multi_indices(d, k), Fk1 = multi_indices(d, k - 1);
  const int nm = (int)Fm.size(), nk = (int)Fk.size(), ng = (int)Fk1.size();
  std::map<MI, int> fm_index;
  for (int j = 0; j < nm; ++j) fm_index[Fm[j]] = j;
  // facet Vandermonde of degree m at the facet lattice points mu = beta / m,
  // and the moment matrices
  std::vector<double> Mkk(nk * nk), Mkm((size_t)nk * nm), Mgg(ng * ng), Mgm((size_t)ng * nm);
  for (int i = 0; i < nk; ++i) {
    for (int j = 0; j < nk; ++j) Mkk[i * nk + j] = simplex_moment2(Fk[i], Fk[j]);
    for (int j = 0; j < nm; ++j) Mkm[(size_t)i * nm + j] = simplex_moment2(Fk[i], Fm[j]);
  }
  for (int i = 0; i < ng; ++i) {
    for (int j = 0; j < ng; ++j) Mgg[i * ng + j] = simplex_moment2(Fk1[i], Fk1[j]);
    for (int j = 0; j < nm; ++j) Mgm[(size_t)i * nm + j] = simplex_moment2(Fk1[i], Fm[j]);
  }
  xD.assign((size_t)pb->ne * s.nd, 0.0);
  std::vector<double> gp((size_t)nm * d), coef((size_t)nm * d);
  for (int64_t e = 0; e < pb->ne; ++e) {
    const int perm = pb->h_elem_perm[e];
    for (int i = 0; i < nv; ++i) {
      if (pb->h_elem_ff[e * nv + i] >= 0) continue;   // free (interior or outlet) facet
      int fv[3], c = 0;
      for (int j = 0; j < nv; ++j)
        if (j != i) fv[c++] = j;
      double X[3][3] = {};
      for (int j = 0; j < d; ++j)
        for (int r = 0; r < d; ++r) X[j][r] = pb->h_coords[(size_t)pb->h_elem_verts[e * nv + fv[j]] * d + r];
      double t[2][3] = {}, n[3] = {}, area;
      for (int r = 0; r < d; ++r) {
        t[0][r] = X[1][r] - X[0][r];
        if (d == 3) t[1][r] = X[2][r] - X[0][r];
      }
      if (d == 2) {
        n[0] = t[0][1];
        n[1] = -t[0][0];
      } else {
        n[0] = t[0][1] * t[1][2] - t[0][2] * t[1][1];
        n[1] = t[0][2] * t[1][0] - t[0][0] * t[1][2];
        n[2] = t[0][0] * t[1][1] - t[0][1] * t[1][0];
      }
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      area = d == 2 ? nn : 0.5 * nn;
      for (int r = 0; r < 3; ++r) n[r] /= nn;
      // g at the facet's lattice points (sorted lattice index -> facet index)
      for (int p = 0; p < nlat; ++p) {
        const int sidx = pb->ref.latmap[(size_t)perm * nlat + p];
        const MI& a = Ilat[sidx];
        if (a[i] != 0) continue;
        MI fmi;
        for (int j = 0; j < nv; ++j)
          if (j != i) fmi.push_back(a[j]);
        const int q = fm_index.at(fmi);
        for (int r = 0; r < d; ++r) gp[(size_t)q * d + r] = g_lattice[((size_t)e * nlat + p) * d + r];
      }
      // monomial coefficients of the degree-m interpolant on the facet
      {
        std::vector<double> V((size_t)nm * nm);
        for (int q = 0; q < nm; ++q)
          for (int j = 0; j < nm; ++j) {
            double v = 1.0;
            for (int b = 0; b < d; ++b) v *= std::pow((double)Fm[q][b] / m, Fm[j][b]);
            V[(size_t)q * nm + j] = v;
          }
        for (int r = 0; r < d; ++r) {
          std::vector<double> rhs(nm), Vc = V;
          for (int q = 0; q < nm; ++q) rhs[q] = gp[(size_t)q * d + r];
          solve_dense(Vc, nm, rhs);
          for (int j = 0; j < nm; ++j) coef[(size_t)j * d + r] = rhs[j];
        }
      }
      double* out = &xD[(size_t)e * s.nd + (size_t)i * s.nfb];
      // normal dofs
      {
        std::vector<double> rhs(nk, 0.0), M = Mkk;
        for (int a = 0; a < nk; ++a)
          for (int j = 0; j < nm; ++j) {
            double gn = 0.0;
            for (int r = 0; r < d; ++r) gn += coef[(size_t)j * d + r] * n[r];
            rhs[a] += Mkm[(size_t)a * nm + j] * gn;
          }
        solve_dense(M, nk, rhs);
        for (int a = 0; a < nk; ++a) out[a] = area * rhs[a];
      }
      // tangential dofs: (T (x) M_gg) c = rhs, T_bb' = t_b . t_b'
      {
        const int nt = (d - 1) * ng;
        std::vector<double> M((size_t)nt * nt), rhs(nt, 0.0);
        for (int b = 0; b < d - 1; ++b)
          for (int b2 = 0; b2 < d - 1; ++b2) {
            double tt = 0.0;
            for (int r = 0; r < d; ++r) tt += t[b][r] * t[b2][r];
            for (int g1 = 0; g1 < ng; ++g1)
              for (int g2 = 0; g2 < ng; ++g2) M[(size_t)(b * ng + g1) * nt + b2 * ng + g2] = tt * Mgg[g1 * ng + g2];
          }
        for (int b = 0; b < d - 1; ++b)
          for (int g1 = 0; g1 < ng; ++g1)
            for (int j = 0; j < nm; ++j) {
              double gt = 0.0;
              for (int r = 0; r < d; ++r) gt += coef[(size_t)j * d + r] * t[b][r];
              rhs[b * ng + g1] += Mgm[(size_t)g1 * nm + j] * gt;
            }
        solve_dense(M, nt, rhs);
        for (int q = 0; q < nt; ++q) out[s.nF + q] = rhs[q];
      }
      // k = 1 (Sec. 7): omega's dof, the flux of curl g through F w.r.t.
      // n_F, by Stokes the circulation of g's interpolant along dF
      // (X_0 -> X_1 -> X_2, positive about n_F); on the edge from a to b a
      // facet monomial mu^beta with no weight on the third vertex integrates
      // to beta_a! beta_b! / (beta_a + beta_b + 1)! times (X_b - X_a)
      if (s.nw) {
        double circ = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int b = (a + 1) % 3, o = (a + 2) % 3;
          for (int j = 0; j < nm; ++j) {
            if (Fm[j][o] != 0) continue;
            double gt = 0.0;
            for (int r = 0; r < d; ++r) gt += coef[(size_t)j * d + r] * (X[b][r] - X[a][r]);
            circ += fact(Fm[j][a]) * fact(Fm[j][b]) / fact(Fm[j][a] + Fm[j][b] + 1) * gt;
          }
        }
        out[s.nF + s.nh] = circ;
      }
    }
  }
}

}  // namespace mcs
