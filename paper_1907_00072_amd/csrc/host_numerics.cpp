// Host-side dense numerics for the polynomial build.
//
// * harmonic_ritz: the zeros of the GMRES residual polynomial after s Arnoldi
//   steps are the harmonic Ritz values, the eigenvalues of
//   H_s + h_{s+1,s}^2 H_s^{-T} e_s e_s^T (the rank-one term only changes the
//   last column, so the matrix stays upper Hessenberg).
// * hessenberg_eigvals: Francis implicit double-shift QR on a Hessenberg
//   matrix (Golub & Van Loan, Matrix Computations, Sec. 7.5), eigenvalues only:
//   transformations are confined to the active unreduced window, 3x3 and 2x2
//   Householder reflectors chase the bulge, small subdiagonals deflate, and
//   1x1 / 2x2 blocks give the eigenvalues.
// * leja_order: modified Leja ordering (Bai, Hu & Reichel 1994) with conjugate
//   pairs kept adjacent, so that the product form of the polynomial is evaluated
//   stably at high degree.
#include "host_numerics.h"

#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <cmath>
#include <numeric>

#include "../../include/pp.h"

namespace ppn {

namespace {

// Eigenvalues of [[a, b], [c, d]]; a complex pair is returned as exact conjugates.
void eig2x2(double a, double b, double c, double d, double *r1, double *i1, double *r2,
            double *i2) {
  const double p = 0.5 * (a - d);
  const double bc = b * c;
  const double disc = p * p + bc;
  if (disc >= 0.0) {
    const double sq = std::sqrt(disc);
    const double z = p + std::copysign(sq, p);
    if (z == 0.0) {
      *r1 = *r2 = d + p;
    } else {
      *r1 = d + z;
      *r2 = d - bc / z;
    }
    *i1 = *i2 = 0.0;
  } else {
    const double re = d + p;
    const double im = std::sqrt(-disc);
    *r1 = *r2 = re;
    *i1 = im;
    *i2 = -im;
  }
}

// Householder reflector P = I - tau v v^T with v(0) = 1 mapping x to (beta, 0, ...).
// Returns false when x(1..) is already zero (P = I).
bool house(int len, const double *x, double *v, double *tau) {
  double tail = 0.0;
  for (int k = 1; k < len; ++k) tail = std::hypot(tail, x[k]);
  if (tail == 0.0) return false;
  const double alpha = std::hypot(x[0], tail);
  const double beta = (x[0] >= 0.0) ? -alpha : alpha;
  const double v0 = x[0] - beta;
  v[0] = 1.0;
  for (int k = 1; k < len; ++k) v[k] = x[k] / v0;
  *tau = (beta - x[0]) / beta;
  return true;
}

}  // namespace

int hessenberg_eigvals(int s, double *H, double *wr, double *wi) {
  auto h = [&](int i, int j) -> double & { return H[i + (size_t)j * s]; };
  double anorm = 0.0;
  for (int j = 0; j < s; ++j)
    for (int i = 0; i <= std::min(j + 1, s - 1); ++i) anorm += std::fabs(h(i, j));
  if (!std::isfinite(anorm)) return PP_ERR_SINGULAR;
  int u = s - 1;
  int its = 0, total = 0;
  const int max_total = 60 * std::max(s, 1);
  while (u >= 0) {
    // deflation: find the start l of the unreduced block ending at u
    int l = u;
    while (l > 0) {
      double sc = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (sc == 0.0) sc = anorm;
      if (std::fabs(h(l, l - 1)) <= DBL_EPSILON * sc) {
        h(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == u) {
      wr[u] = h(u, u);
      wi[u] = 0.0;
      --u;
      its = 0;
      continue;
    }
    if (l == u - 1) {
      eig2x2(h(u - 1, u - 1), h(u - 1, u), h(u, u - 1), h(u, u), &wr[u - 1], &wi[u - 1],
             &wr[u], &wi[u]);
      u -= 2;
      its = 0;
      continue;
    }
    if (++total > max_total) return PP_ERR_EIG;
    ++its;
    // shifts: the two eigenvalues of the trailing 2x2 block (sum ss, product tt),
    // replaced by ad-hoc values every 10 iterations to break cycles
    double ss, tt;
    if (its % 10 == 0) {
      const double w = std::fabs(h(u, u - 1)) + std::fabs(h(u - 1, u - 2));
      ss = 1.5 * w;
      tt = w * w;
    } else {
      ss = h(u - 1, u - 1) + h(u, u);
      tt = h(u - 1, u - 1) * h(u, u) - h(u - 1, u) * h(u, u - 1);
    }
    // first column of H^2 - ss H + tt I, rows l .. l+2
    double x[3];
    x[0] = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - ss * h(l, l) + tt;
    x[1] = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - ss);
    x[2] = h(l + 2, l + 1) * h(l + 1, l);
    for (int k = l; k <= u - 2; ++k) {
      double v[3], tau;
      if (house(3, x, v, &tau)) {
        const int q = std::max(l, k - 1);
        for (int j = q; j <= u; ++j) {
          const double p = tau * (h(k, j) + v[1] * h(k + 1, j) + v[2] * h(k + 2, j));
          h(k, j) -= p;
          h(k + 1, j) -= p * v[1];
          h(k + 2, j) -= p * v[2];
        }
        if (k > l) {
          h(k + 1, k - 1) = 0.0;
          h(k + 2, k - 1) = 0.0;
        }
        const int r = std::min(k + 3, u);
        for (int i = l; i <= r; ++i) {
          const double p = tau * (h(i, k) + v[1] * h(i, k + 1) + v[2] * h(i, k + 2));
          h(i, k) -= p;
          h(i, k + 1) -= p * v[1];
          h(i, k + 2) -= p * v[2];
        }
      }
      x[0] = h(k + 1, k);
      x[1] = h(k + 2, k);
      x[2] = (k < u - 2) ? h(k + 3, k) : 0.0;
    }
    // last reflector on rows/columns u-1, u
    {
      double v[2], tau;
      if (house(2, x, v, &tau)) {
        const int k = u - 1;
        for (int j = std::max(l, k - 1); j <= u; ++j) {
          const double p = tau * (h(k, j) + v[1] * h(k + 1, j));
          h(k, j) -= p;
          h(k + 1, j) -= p * v[1];
        }
        if (k - 1 >= l) h(k + 1, k - 1) = 0.0;
        for (int i = l; i <= u; ++i) {
          const double p = tau * (h(i, k) + v[1] * h(i, k + 1));
          h(i, k) -= p;
          h(i, k + 1) -= p * v[1];
        }
      }
    }
  }
  for (int i = 0; i < s; ++i)
    if (!std::isfinite(wr[i]) || !std::isfinite(wi[i])) return PP_ERR_EIG;
  return 0;
}

int harmonic_ritz(const double *Hbar, int ldh, int s, std::vector<double> &wr,
                  std::vector<double> &wi) {
  if (s < 1 || ldh < s + 1) return PP_ERR_ARG;
  // solve H_s^T f = e_s by Gaussian elimination with partial pivoting
  std::vector<double> T((size_t)s * s);  // T = H_s^T, column-major
  for (int j = 0; j < s; ++j)
    for (int i = 0; i < s; ++i) T[i + (size_t)j * s] = Hbar[j + (size_t)i * ldh];
  std::vector<double> f(s, 0.0);
  f[s - 1] = 1.0;
  for (int k = 0; k < s; ++k) {
    int piv = k;
    double big = std::fabs(T[k + (size_t)k * s]);
    for (int i = k + 1; i < s; ++i)
      if (std::fabs(T[i + (size_t)k * s]) > big) {
        big = std::fabs(T[i + (size_t)k * s]);
        piv = i;
      }
    if (big == 0.0 || !std::isfinite(big)) return PP_ERR_SINGULAR;
    if (piv != k) {
      for (int j = 0; j < s; ++j) std::swap(T[k + (size_t)j * s], T[piv + (size_t)j * s]);
      std::swap(f[k], f[piv]);
    }
    for (int i = k + 1; i < s; ++i) {
      const double lik = T[i + (size_t)k * s] / T[k + (size_t)k * s];
      if (lik == 0.0) continue;
      for (int j = k; j < s; ++j) T[i + (size_t)j * s] -= lik * T[k + (size_t)j * s];
      f[i] -= lik * f[k];
    }
  }
  for (int k = s - 1; k >= 0; --k) {
    double acc = f[k];
    for (int j = k + 1; j < s; ++j) acc -= T[k + (size_t)j * s] * f[j];
    f[k] = acc / T[k + (size_t)k * s];
  }
  const double hs = Hbar[s + (size_t)(s - 1) * ldh];
  std::vector<double> M((size_t)s * s);
  for (int j = 0; j < s; ++j)
    for (int i = 0; i < s; ++i) M[i + (size_t)j * s] = (i <= j + 1) ? Hbar[i + (size_t)j * ldh] : 0.0;
  for (int i = 0; i < s; ++i) M[i + (size_t)(s - 1) * s] += hs * hs * f[i];
  wr.assign(s, 0.0);
  wi.assign(s, 0.0);
  int rc = hessenberg_eigvals(s, M.data(), wr.data(), wi.data());
  if (rc) return rc;
  for (int i = 0; i < s; ++i)
    if (wr[i] == 0.0 && wi[i] == 0.0) return PP_ERR_SINGULAR;
  return 0;
}

int leja_order(const std::vector<double> &wr, const std::vector<double> &wi,
               std::vector<double> &or_, std::vector<double> &oi) {
  const int s = (int)wr.size();
  int npos = 0, nneg = 0;
  std::vector<int> cand;
  for (int i = 0; i < s; ++i) {
    if (wi[i] > 0) ++npos;
    if (wi[i] < 0) ++nneg;
    if (wi[i] >= 0) cand.push_back(i);
  }
  if (npos != nneg) return PP_ERR_ARG;
  std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
    return wr[a] < wr[b] || (wr[a] == wr[b] && wi[a] < wi[b]);
  });
  or_.clear();
  oi.clear();
  if (cand.empty()) return 0;
  auto take = [&](size_t pos) {
    const int i = cand[pos];
    cand.erase(cand.begin() + pos);
    or_.push_back(wr[i]);
    oi.push_back(wi[i]);
    if (wi[i] > 0) {
      or_.push_back(wr[i]);
      oi.push_back(-wi[i]);
    }
  };
  // start: largest modulus; ties larger Re, then Im > 0
  size_t best = 0;
  for (size_t p = 1; p < cand.size(); ++p) {
    const int a = cand[p], b = cand[best];
    const double ma = std::hypot(wr[a], wi[a]), mb = std::hypot(wr[b], wi[b]);
    const bool better = ma > mb || (ma == mb && (wr[a] > wr[b] ||
                                                 (wr[a] == wr[b] && (wi[a] > 0) && !(wi[b] > 0))));
    if (better) best = p;
  }
  take(best);
  while (!cand.empty()) {
    size_t bp = 0;
    double bs = 0.0;
    for (size_t p = 0; p < cand.size(); ++p) {
      const int i = cand[p];
      double sc = 0.0;
      for (size_t k = 0; k < or_.size(); ++k) {
        const double dist = std::hypot(wr[i] - or_[k], wi[i] - oi[k]);
        if (dist == 0.0) {
          sc = -INFINITY;
          break;
        }
        sc += std::log(dist);
      }
      if (p == 0 || sc > bs) {
        bp = p;
        bs = sc;
      }
    }
    take(bp);
  }
  return 0;
}

int step_table(const std::vector<double> &re, const std::vector<double> &im,
               std::vector<Step> &steps) {
  steps.clear();
  const size_t d = re.size();
  for (size_t k = 0; k < d; ++k) {
    if (!std::isfinite(re[k]) || !std::isfinite(im[k])) return PP_ERR_SINGULAR;
    if (im[k] == 0.0) {
      if (re[k] == 0.0) return PP_ERR_SINGULAR;
      steps.push_back({0, 1.0 / re[k], 0.0});
    } else {
      if (!(im[k] > 0) || k + 1 >= d || re[k + 1] != re[k] || im[k + 1] != -im[k])
        return PP_ERR_ARG;
      const double m2 = re[k] * re[k] + im[k] * im[k];
      if (!(m2 > 0) || !std::isfinite(m2)) return PP_ERR_SINGULAR;
      steps.push_back({1, 2.0 * re[k] / m2, 1.0 / m2});
      ++k;
    }
  }
  return 0;
}

int cholesky_upper(const double *G, int ldg, int k, std::vector<double> &R) {
  R.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i <= j; ++i) {
      double acc = G[i + (size_t)j * ldg];
      for (int q = 0; q < i; ++q) acc -= R[q + (size_t)i * k] * R[q + (size_t)j * k];
      if (i < j) {
        R[i + (size_t)j * k] = acc / R[i + (size_t)i * k];
      } else {
        if (!(acc > 0.0)) return j + 1;
        R[j + (size_t)j * k] = std::sqrt(acc);
      }
    }
  }
  return 0;
}

void cholesky_solve(const std::vector<double> &R, int k, const double *rhs, double *y) {
  std::vector<double> z(k);
  for (int i = 0; i < k; ++i) {  // R^T z = rhs
    double acc = rhs[i];
    for (int q = 0; q < i; ++q) acc -= R[q + (size_t)i * k] * z[q];
    z[i] = acc / R[i + (size_t)i * k];
  }
  for (int i = k - 1; i >= 0; --i) {  // R y = z
    double acc = z[i];
    for (int q = i + 1; q < k; ++q) acc -= R[i + (size_t)q * k] * y[q];
    y[i] = acc / R[i + (size_t)i * k];
  }
}

void slab_order(int ntile, int S, int w, int K, int group, std::vector<SlabPart> &out) {
  out.clear();
  S = std::max(S, 1);
  w = std::max(w, 0);
  group = std::max(group, 1);
  for (int k0 = 0; k0 < K; k0 += group) {
    const int k1 = std::min(K, k0 + group);
    const int64_t span = (int64_t)ntile + (int64_t)(k1 - 1 - k0) * w;
    for (int64_t b = 0; b * S < span; ++b) {
      for (int k = k0; k < k1; ++k) {
        const int64_t shift = (int64_t)(k - k0) * w;
        const int t0 = (int)std::max<int64_t>(0, b * S - shift);
        const int t1 = (int)std::min<int64_t>(ntile, (b + 1) * S - shift);
        if (t1 > t0) out.push_back(SlabPart{k, t0, t1});
      }
    }
  }
}

}  // namespace ppn
