// Model construction for the general LBGK model (Sec. II and Sec. III of
// Shi, He and Guo).  See coeffs.hpp.
//
// Routes chosen here (the CPU test oracle takes other ones, so the two can be
// compared):
//  * tau_k are read off the power series of g(s) = u / (1 + tau u),
//    u = e^s - 1, the generating function of the relaxation polynomials of
//    eq. (taus);
//  * the integrand of Pi_k0 is the binomial pattern common to eqs. (Pi4),
//    (Pi5), (Pi6):  (Pi_1')^k + sum_{r=2}^{k-1} C(k,r) beta_r Pi_r' (Pi_1')^{k-r}
//    + A_k0;
//  * M_q^{-1} is obtained by Gauss-Jordan elimination of the moment
//    (Vandermonde) matrix M[k][j] = e_j^k of Sec. III.A/B.
#include "coeffs.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace lbm {

// Odd q puts the rest velocity first; even q (D1Q4, D1Q6, Sec. III) has none.
int lattice_velocity(int q, int j) {
  static const int odd[kMaxQ] = {0, 1, -1, 2, -2, 3, -3};
  static const int even[kMaxQ] = {1, -1, 2, -2, 3, -3, 0};
  return (q & 1) ? odd[j] : even[j];
}

namespace {

using qf = __float128;
using QPoly = std::vector<qf>;   // ascending powers of phi

QPoly trim(QPoly p) {
  while (!p.empty() && p.back() == 0) p.pop_back();
  return p;
}

QPoly add(const QPoly& a, const QPoly& b) {
  QPoly r(a.size() > b.size() ? a.size() : b.size(), 0);
  for (size_t i = 0; i < a.size(); ++i) r[i] += a[i];
  for (size_t i = 0; i < b.size(); ++i) r[i] += b[i];
  return trim(r);
}

QPoly scale(const QPoly& a, qf s) {
  QPoly r(a.size());
  for (size_t i = 0; i < a.size(); ++i) r[i] = a[i] * s;
  return trim(r);
}

QPoly mul(const QPoly& a, const QPoly& b) {
  if (a.empty() || b.empty()) return {};
  QPoly r(a.size() + b.size() - 1, 0);
  for (size_t i = 0; i < a.size(); ++i)
    for (size_t j = 0; j < b.size(); ++j) r[i + j] += a[i] * b[j];
  return trim(r);
}

QPoly power(const QPoly& a, int n) {
  QPoly r{1};
  for (int i = 0; i < n; ++i) r = mul(r, a);
  return r;
}

QPoly deriv(const QPoly& a) {
  QPoly r;
  for (size_t i = 1; i < a.size(); ++i) r.push_back(a[i] * (qf)i);
  return trim(r);
}

QPoly antideriv(const QPoly& a) {   // vanishes at phi = 0
  QPoly r(a.size() + 1, 0);
  for (size_t i = 0; i < a.size(); ++i) r[i + 1] = a[i] / (qf)(i + 1);
  return trim(r);
}

QPoly constant(const QPoly*, qf v) { return trim(QPoly{v}); }
QPoly identity(const QPoly*) { return QPoly{0, 1}; }

// Power sums with real exponents, sum_i c_i phi^{g_i} (exponents >= 0): the
// closure of the operations the auxiliary moments need when Pi_k carries real
// powers (Sec. III.C).  Terms sorted by exponent, no zero coefficients.
struct GPoly {
  std::vector<std::pair<qf, qf>> t;   // (exponent, coefficient)
};

GPoly normal(std::vector<std::pair<qf, qf>> v) {
  std::sort(v.begin(), v.end(),
            [](const std::pair<qf, qf>& a, const std::pair<qf, qf>& b) { return a.first < b.first; });
  GPoly r;
  for (const auto& e : v) {
    if (!r.t.empty() && r.t.back().first == e.first)
      r.t.back().second += e.second;
    else
      r.t.push_back(e);
  }
  GPoly o;
  for (const auto& e : r.t)
    if (e.second != 0) o.t.push_back(e);
  return o;
}

GPoly add(const GPoly& a, const GPoly& b) {
  std::vector<std::pair<qf, qf>> v = a.t;
  v.insert(v.end(), b.t.begin(), b.t.end());
  return normal(v);
}

GPoly scale(const GPoly& a, qf s) {
  std::vector<std::pair<qf, qf>> v;
  for (const auto& e : a.t) v.push_back({e.first, e.second * s});
  return normal(v);
}

GPoly mul(const GPoly& a, const GPoly& b) {
  std::vector<std::pair<qf, qf>> v;
  for (const auto& x : a.t)
    for (const auto& y : b.t) v.push_back({x.first + y.first, x.second * y.second});
  return normal(v);
}

GPoly power(const GPoly& a, int n) {
  GPoly r;
  r.t.push_back({0, 1});
  for (int i = 0; i < n; ++i) r = mul(r, a);
  return r;
}

GPoly deriv(const GPoly& a) {
  std::vector<std::pair<qf, qf>> v;
  for (const auto& e : a.t)
    if (e.first != 0) v.push_back({e.first - 1, e.second * e.first});
  return normal(v);
}

GPoly antideriv(const GPoly& a) {   // vanishes at phi = 0 (exponents >= 0)
  std::vector<std::pair<qf, qf>> v;
  for (const auto& e : a.t) v.push_back({e.first + 1, e.second / (e.first + 1)});
  return normal(v);
}

GPoly constant(const GPoly*, qf v) {
  GPoly r;
  if (v != 0) r.t.push_back({0, v});
  return r;
}
GPoly identity(const GPoly*) {
  GPoly r;
  r.t.push_back({1, 1});
  return r;
}

qf floorq(qf x) {   // exponents here are small and non-negative
  qf f = (qf)(long long)x;
  return f > x ? f - 1 : f;
}

qf qabs(qf x) { return x < 0 ? -x : x; }

// tau_1..tau_6: coefficients of s^k in u/(1 + tau u) = sum_{r>=1} (-tau)^{r-1} u^r
void relaxation_series(qf tau, qf out[7]) {
  const int K = 6;
  qf u[K + 1] = {0};
  qf fact = 1;
  for (int n = 1; n <= K; ++n) {
    fact *= n;
    u[n] = 1 / fact;
  }
  qf g[K + 1] = {0};
  qf ur[K + 1] = {0};   // u^r, truncated
  ur[0] = 1;
  qf coef = 1;          // (-tau)^{r-1}
  for (int r = 1; r <= K; ++r) {
    qf next[K + 1] = {0};
    for (int i = 0; i <= K; ++i)
      for (int j = 1; i + j <= K; ++j) next[i + j] += ur[i] * u[j];
    std::memcpy(ur, next, sizeof(ur));
    for (int k = 0; k <= K; ++k) g[k] += coef * ur[k];
    coef *= -tau;
  }
  for (int k = 0; k <= K; ++k) out[k] = g[k];
}

bool finite_d(double v) { return std::isfinite(v); }

long long binom(int n, int k) {
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// M[k][j] = e_j^k, inverted by Gauss-Jordan with partial pivoting
bool invert_moment_matrix(int q, qf inv[kMaxQ][kMaxQ]) {
  qf a[kMaxQ][2 * kMaxQ];
  for (int k = 0; k < q; ++k) {
    for (int j = 0; j < q; ++j) {
      qf v = 1;
      for (int p = 0; p < k; ++p) v *= lattice_velocity(q, j);
      a[k][j] = v;
      a[k][q + j] = (k == j) ? 1 : 0;
    }
  }
  for (int col = 0; col < q; ++col) {
    int piv = col;
    for (int r = col + 1; r < q; ++r)
      if (qabs(a[r][col]) > qabs(a[piv][col])) piv = r;
    if (a[piv][col] == 0) return false;
    if (piv != col)
      for (int j = 0; j < 2 * q; ++j) {
        qf t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
    qf p = a[col][col];
    for (int j = 0; j < 2 * q; ++j) a[col][j] /= p;
    for (int r = 0; r < q; ++r) {
      if (r == col || a[r][col] == 0) continue;
      qf f = a[r][col];
      for (int j = 0; j < 2 * q; ++j) a[r][j] -= f * a[col][j];
    }
  }
  for (int r = 0; r < q; ++r)
    for (int j = 0; j < q; ++j) inv[r][j] = a[r][q + j];
  return true;
}

constexpr double kSingular = 1e-10;   // |tau_k| below this is treated as a root

// Pi_k0 = int_0^phi I_k, k = 2..q-1, with the integrand pattern of eqs. (Pi4),
// (Pi5), (Pi6), and the scaled moments Pi_bar_k (Sec. III.A/B), for
// polynomials (QPoly) and real-exponent power sums (GPoly) alike
template <class P>
void scaled_moments(const P Pi[7], const qf beta[7], const qf A[7], bool corrected, int q, qf c, int scheme,
                    P Pbar[kMaxQ]) {
  const P* tag = nullptr;
  const P d1 = deriv(Pi[1]);
  P d1pow[7];
  for (int p = 0; p <= 6; ++p) d1pow[p] = power(d1, p);
  P Pi0[7];
  for (int k = 2; k < q; ++k) {
    P I = d1pow[k];
    for (int r = 2; r <= k - 1; ++r) {
      P lead = scale(deriv(Pi[r]), beta[r]);
      if (corrected && (r == 4 || r == 5)) lead = add(lead, constant(tag, A[r]));
      I = add(I, scale(mul(lead, d1pow[k - r]), (qf)binom(k, r)));
    }
    if (k >= 4) I = add(I, constant(tag, A[k]));
    Pi0[k] = antideriv(I);
  }
  Pbar[0] = identity(tag);
  Pbar[1] = scale(Pi[1], 1 / c);
  qf ck = c;
  for (int k = 2; k < q; ++k) {
    ck *= c;
    Pbar[k] = scale(add(Pi0[k], scale(Pi[k], beta[k])), 1 / ck);
  }
  if (scheme == 2) Pbar[q - 1] = P();
}

// Exponents closer than this are evaluated with one fractional part: sums of
// binary inputs that stand for the same fraction (3 * 1/3 next to 1, 4/3 next
// to 1 + 1/3) differ by a few units in the last place; the power then changes
// by at most kGTol * |ln phi| relative.
constexpr double kGTol = 1e-13;

// class (fractional part) and integer degree of exponent g: g ~ nu[c] + d
void split_exponent(qf g, std::vector<qf>* nus, int* cls, int* deg) {
  qf r = floorq(g + (qf)0.5);
  if (qabs(g - r) <= kGTol) {
    *cls = 0;
    *deg = (int)r;
    return;
  }
  const qf fl = floorq(g), fr = g - fl;
  *deg = (int)fl;
  for (size_t c = 1; c < nus->size(); ++c)
    if (qabs((*nus)[c] - fr) <= kGTol) {
      *cls = (int)c;
      return;
    }
  nus->push_back(fr);
  *cls = (int)nus->size() - 1;
}

// f_eq_j = sum_k M^{-1}[j][k] Pi_bar_k as power sums, sorted into classes by
// the fractional part of the exponent: phi^g = phi^nu phi^d, nu = g - floor(g)
lbm_status collapse_general(const GPoly Pbar[kMaxQ], const qf inv[kMaxQ][kMaxQ], int q, qf omega, Model* mdl) {
  GPoly G[kMaxQ];
  std::vector<qf> nus{0};
  for (int j = 0; j < q; ++j) {
    for (int k = 0; k < q; ++k) G[j] = add(G[j], scale(Pbar[k], inv[j][k]));
    for (const auto& e : G[j].t) {
      int c, dg;
      split_exponent(e.first, &nus, &c, &dg);
      if (dg > kGDeg) return LBM_ERR_UNSUPPORTED;
    }
  }
  if ((int)nus.size() > kGClasses) return LBM_ERR_UNSUPPORTED;
  std::sort(nus.begin() + 1, nus.end());
  mdl->gF = (int)nus.size();
  int D = 1;
  for (int c = 0; c < mdl->gF; ++c) {
    mdl->gnuq[c] = nus[c];
    mdl->gnu[c] = (double)nus[c];
  }
  for (int j = 0; j < q; ++j) {
    for (const auto& e : G[j].t) {
      int c, dg;
      split_exponent(e.first, &nus, &c, &dg);
      mdl->gGq[c][j][dg] += e.second;
      D = std::max(D, dg);
    }
  }
  mdl->D = D;
  for (int c = 0; c < mdl->gF; ++c) {
    // lowest nonzero degree and the gcd of the gaps above it (e.g. phi^(3/2)
    // fluxes give degrees 1, 4, 7 in the integer class: a polynomial in phi^3)
    int lo = -1, hi = 0, step = 0;
    for (int dg = 0; dg <= kGDeg; ++dg) {
      bool nz = false;
      for (int j = 0; j < q; ++j) nz = nz || mdl->gGq[c][j][dg] != 0;
      if (!nz) continue;
      if (lo < 0)
        lo = dg;
      else
        step = std::gcd(step, dg - lo);
      hi = dg;
    }
    if (lo < 0) lo = hi = 0;
    if (step == 0) step = 1;
    mdl->gd0[c] = lo;
    mdl->gstep[c] = step;
    mdl->gK[c] = (hi - lo) / step + 1;
  }
  for (int c = 0; c < mdl->gF; ++c)
    for (int j = 0; j < q; ++j)
      for (int dg = 0; dg <= kGDeg; ++dg) {
        mdl->gG[c][j][dg] = (double)mdl->gGq[c][j][dg];
        mdl->gwG[c][j][dg] = (double)(omega * mdl->gGq[c][j][dg]);
        if (!finite_d(mdl->gG[c][j][dg]) || !finite_d(mdl->gwG[c][j][dg])) return LBM_ERR_SINGULAR_TAU;
      }
  return LBM_OK;
}

}  // namespace

long double general_feq(const Model& m, int j, long double phi) {
  long double acc = 0;
  for (int c = 0; c < m.gF; ++c) {
    long double p = 0;
    for (int dg = kGDeg; dg >= 0; --dg) p = p * phi + (long double)m.gGq[c][j][dg];
    acc += (c == 0 ? 1.0L : powl(phi, (long double)m.gnuq[c])) * p;
  }
  return acc;
}

long double general_dfeq(const Model& m, int j, long double phi) {
  long double acc = 0;
  for (int c = 0; c < m.gF; ++c)
    for (int dg = 0; dg <= kGDeg; ++dg) {
      const long double g = (long double)m.gnuq[c] + dg;
      const long double v = (long double)m.gGq[c][j][dg];
      if (v != 0 && g != 0) acc += v * g * powl(phi, g - 1);
    }
  return acc;
}

int resolved_order(const lbm_desc& d) {
  int top = 1;
  for (int k = 2; k <= 6; ++k)
    if (d.alpha[k] != 0.0 && (d.pi_deg[k] >= 0 || d.pi_terms[k] > 0)) top = k;
  if (d.m == 0) return top;
  if (d.m < 1 || d.m > 6 || d.m < top) return 0;
  return d.m;
}

int resolved_lattice(const lbm_desc& d) {
  int m = resolved_order(d);
  if (m == 0) return 0;
  if (d.q == 0) return m <= 4 ? 5 : 7;
  if (d.q < 4 || d.q > 7 || d.q < m + 1) return 0;
  return d.q;
}

lbm_status build_model(const lbm_desc& d, Model* out) {
  // ---- validation (host, before any device work) ----
  if (!out) return LBM_ERR_INVALID_ARG;
  if (d.scheme < 0 || d.scheme > 2 || (d.am != LBM_AM_CORRECTED && d.am != LBM_AM_PAPER))
    return LBM_ERR_INVALID_ARG;
  if (d.prec != LBM_F64 && d.prec != LBM_F32_DEV && d.prec != LBM_F32_DEV_ARITH32) return LBM_ERR_INVALID_ARG;
  if (d.bc != LBM_BC_PERIODIC && d.bc != LBM_BC_DIRICHLET_EQ && d.bc != LBM_BC_DIRICHLET_NEE)
    return LBM_ERR_INVALID_ARG;
  for (int k = 1; k <= 6; ++k) {
    if (d.pi_deg[k] < -1 || d.pi_deg[k] > 4) return LBM_ERR_INVALID_ARG;
    for (int p = 0; p <= d.pi_deg[k]; ++p)
      if (!finite_d(d.pi_coef[k][p])) return LBM_ERR_INVALID_ARG;
    if (d.pi_terms[k] < 0 || d.pi_terms[k] > 4) return LBM_ERR_INVALID_ARG;
    for (int i = 0; i < d.pi_terms[k]; ++i) {
      const double e = d.pi_gexp[k][i];
      if (!finite_d(e) || !finite_d(d.pi_gcoef[k][i]) || !(e == 0.0 || (e >= 1.0 && e <= 8.0)))
        return LBM_ERR_INVALID_ARG;
    }
    if (!finite_d(d.alpha[k])) return LBM_ERR_INVALID_ARG;
  }
  if (!(d.dx > 0) || !(d.dt > 0) || !finite_d(d.dx) || !finite_d(d.dt)) return LBM_ERR_INVALID_ARG;
  if (!(d.tau > 0.5) || !finite_d(d.tau)) return LBM_ERR_INVALID_ARG;
  const int m = resolved_order(d);
  const int q = resolved_lattice(d);
  if (m == 0 || q == 0) return LBM_ERR_INVALID_ARG;
  if (d.n < q || d.n > (int64_t(1) << 30)) return LBM_ERR_INVALID_ARG;

  Model mdl;
  mdl.q = q;
  mdl.m = m;
  mdl.scheme = d.scheme == 2 ? 2 : 1;
  mdl.tau = d.tau;
  const qf dx = d.dx, dt = d.dt, tau = d.tau;
  const qf c = dx / dt;
  mdl.c = (double)c;

  // ---- relaxation polynomials (eq. taus) ----
  qf tk[7];
  relaxation_series(tau, tk);

  // ---- Pi_k: polynomials, or power sums when a given exponent is not an
  // integer in 0..4 ----
  QPoly Pi[7];
  GPoly gPi[7];
  bool general = false;
  for (int k = 1; k <= 6; ++k) {
    std::vector<std::pair<qf, qf>> v;
    if (d.pi_terms[k] > 0) {
      for (int i = 0; i < d.pi_terms[k]; ++i) {
        const qf e = d.pi_gexp[k][i];
        if (e != floorq(e) || e > 4) general = true;
        v.push_back({e, (qf)d.pi_gcoef[k][i]});
      }
    } else {
      for (int i = 0; i <= d.pi_deg[k]; ++i) v.push_back({(qf)i, (qf)d.pi_coef[k][i]});
    }
    gPi[k] = normal(v);
  }
  for (int k = 1; k <= 6 && !general; ++k) {
    QPoly p;
    for (const auto& e : gPi[k].t) {
      const int i = (int)e.first;
      if ((int)p.size() <= i) p.resize(i + 1, 0);
      p[i] += e.second;
    }
    Pi[k] = trim(p);
  }

  // ---- beta_k = alpha_k / (dt^{k-1} tau_k), zero where alpha_k = 0 ----
  qf beta[7] = {0};
  for (int k = 2; k <= 6; ++k) {
    if (k > m || d.alpha[k] == 0.0 || gPi[k].t.empty()) continue;
    if (qabs(tk[k]) < kSingular) return LBM_ERR_SINGULAR_TAU;
    qf dtp = 1;
    for (int i = 0; i < k - 1; ++i) dtp *= dt;
    beta[k] = (qf)d.alpha[k] / (dtp * tk[k]);
  }

  // ---- corrections A_40, A_50, A_60 ----
  const qf t2 = tk[2], t3 = tk[3], t4 = tk[4], t5 = tk[5], t6 = tk[6];
  const bool corrected = d.am == LBM_AM_CORRECTED;
  qf A[7] = {0};
  if (q > 4) {
    qf num = t2 * (3 * t3 - t2 * t2) * beta[2] * beta[2];
    if (num != 0) {
      if (qabs(t4) < kSingular) return LBM_ERR_SINGULAR_TAU;
      A[4] = num / t4;
    }
  }
  if (q > 5) {
    qf num = (4 * t2 * t4 + 3 * t3 * t3 - 2 * t2 * t2 * t3) * beta[2] * beta[3];
    if (num != 0) {
      if (qabs(t5) < kSingular) return LBM_ERR_SINGULAR_TAU;
      A[5] = num / t5;
    }
  }
  if (q > 6) {
    qf num = (5 * t2 * t5 + 3 * t3 * t4 - 2 * t2 * t2 * t4) * beta[2] * beta[4] +
             (4 * t4 - t2 * t3) * t3 * beta[3] * beta[3] +
             (t2 * t3 - 6 * t4) * t2 * t2 * beta[2] * beta[2] * beta[2];
    if (corrected) num += 5 * t2 * t5 * beta[2] * A[4];
    if (num != 0) {
      if (qabs(t6) < kSingular) return LBM_ERR_SINGULAR_TAU;
      A[6] = num / t6;
    }
  }

  qf inv[kMaxQ][kMaxQ];
  if (!invert_moment_matrix(q, inv)) return LBM_ERR_INVALID_ARG;
  const qf omega = 1 / tau;
  mdl.w0 = (double)(1 - omega);
  if (general) {
    if (d.prec == LBM_F32_DEV_ARITH32) return LBM_ERR_UNSUPPORTED;
    GPoly Pbar[kMaxQ];
    scaled_moments(gPi, beta, A, corrected, q, c, mdl.scheme, Pbar);
    lbm_status st = collapse_general(Pbar, inv, q, omega, &mdl);
    if (st != LBM_OK) return st;
    set_rest_state(&mdl, 0.0);
    *out = mdl;
    return LBM_OK;
  }

  // ---- auxiliary moments and scaled moments (Sec. II.C-F, III.A/B) ----
  QPoly Pbar[kMaxQ];
  scaled_moments(Pi, beta, A, corrected, q, c, mdl.scheme, Pbar);

  // ---- collapse f_eq = M_q^{-1} Pi_bar into polynomials in phi ----
  int D = 1;
  for (int k = 0; k < q; ++k)
    if ((int)Pbar[k].size() - 1 > D) D = (int)Pbar[k].size() - 1;
  if (D > kMaxDeg) return LBM_ERR_UNSUPPORTED;
  mdl.D = D;
  for (int j = 0; j < q; ++j) {
    for (int p = 0; p <= D; ++p) {
      qf g = 0;
      for (int k = 0; k < q; ++k)
        if (p < (int)Pbar[k].size()) g += inv[j][k] * Pbar[k][p];
      mdl.Gq[j][p] = g;
      mdl.G[j][p] = (double)g;
      mdl.wG[j][p] = (double)(omega * g);
      if (!finite_d(mdl.G[j][p]) || !finite_d(mdl.wG[j][p])) return LBM_ERR_SINGULAR_TAU;
    }
  }
  set_rest_state(&mdl, 0.0);
  *out = mdl;
  return LBM_OK;
}

void set_rest_state(Model* mdl, double phi_rest) {
  const qf r = phi_rest;
  const qf omega = 1 / (qf)mdl->tau;
  mdl->phi_rest = phi_rest;
  if (mdl->gF > 0) {   // power sums: f_rest only (the relaxation stays in phi)
    for (int j = 0; j < mdl->q; ++j) {
      const long double h = general_feq(*mdl, j, (long double)phi_rest);
      mdl->f_rest[j] = (double)h;
      mdl->wfrest[j] = (double)((long double)omega * h);
    }
    return;
  }
  for (int j = 0; j < mdl->q; ++j) {
    // Taylor shift: f_eq_j(r + delta) = sum_p H[j][p] delta^p, H[j][p] = sum_k C(k,p) G[j][k] r^{k-p}
    for (int p = 0; p <= mdl->D; ++p) {
      qf h = 0;
      qf rp = 1;
      for (int k = p; k <= mdl->D; ++k) {
        h += (qf)binom(k, p) * mdl->Gq[j][k] * rp;
        rp *= r;
      }
      if (p == 0) {
        mdl->f_rest[j] = (double)h;
        mdl->wfrest[j] = (double)(omega * h);
        mdl->wG0rest[j] = (double)(omega * (mdl->Gq[j][0] - h));
        mdl->H[j][0] = 0.0;
        mdl->wH[j][0] = 0.0;
      } else {
        mdl->H[j][p] = (double)h;
        mdl->wH[j][p] = (double)(omega * h);
      }
    }
  }
}

}  // namespace lbm

// ---------------------------------------------------------------------------
// Linear (von Neumann) stability of the scheme about a uniform state phi_bar:
// f_eq(phi_bar + d) ~ f_eq(phi_bar) + w d with w_j = f_eq_j'(phi_bar), so one
// step acts on a Fourier mode exp(i kappa x) as A = E ((1 - omega) I + omega w 1^T),
// E = diag(exp(-i kappa e_j)).  A is a rank-one update of a diagonal matrix; its
// eigenvalues are the roots of
//   P(lam) = prod_j (lam - c E_j) - omega sum_j E_j w_j prod_{l != j} (lam - c E_l),
// c = 1 - omega, found by Durand-Kerner iteration.
// ---------------------------------------------------------------------------
#include <complex>

namespace lbm {
namespace {
using cld = std::complex<long double>;

// coefficients (ascending) of prod over roots r of (lam - r)
void poly_from_roots(const cld* r, int m, cld* out) {
  for (int i = 0; i <= m; ++i) out[i] = 0;
  out[0] = 1;
  int deg = 0;
  for (int k = 0; k < m; ++k) {
    for (int i = deg + 1; i >= 1; --i) out[i] = out[i - 1] - r[k] * out[i];
    out[0] = -r[k] * out[0];
    ++deg;
  }
}

long double spectral_radius(const Model& m, const long double* w, long double kappa) {
  const int q = m.q;
  const long double omega = 1.0L / (long double)m.tau, c = 1.0L - omega;
  cld E[kMaxQ], P[kMaxQ + 1], T[kMaxQ + 1], r[kMaxQ];
  for (int j = 0; j < q; ++j) E[j] = std::polar(1.0L, -kappa * (long double)lattice_velocity(q, j));
  for (int j = 0; j < q; ++j) r[j] = c * E[j];
  poly_from_roots(r, q, P);
  for (int j = 0; j < q; ++j) {
    cld rr[kMaxQ];
    int k = 0;
    for (int l = 0; l < q; ++l)
      if (l != j) rr[k++] = c * E[l];
    poly_from_roots(rr, q - 1, T);
    for (int i = 0; i < q; ++i) P[i] -= omega * E[j] * w[j] * T[i];
  }
  // Durand-Kerner on the monic polynomial P (degree q)
  cld z[kMaxQ];
  const cld seed(0.4L, 0.9L);
  cld zz = 1;
  for (int i = 0; i < q; ++i) {
    z[i] = zz * 1.1L;
    zz *= seed;
  }
  for (int it = 0; it < 500; ++it) {
    long double move = 0;
    for (int i = 0; i < q; ++i) {
      cld num = P[q];
      for (int d = q - 1; d >= 0; --d) num = num * z[i] + P[d];
      cld den = 1;
      for (int j = 0; j < q; ++j)
        if (j != i) den *= (z[i] - z[j]);
      if (std::abs(den) == 0) den = 1e-30L;
      const cld dz = num / den;
      z[i] -= dz;
      move = std::max(move, std::abs(dz));
    }
    if (move < 1e-15L) break;
  }
  long double rad = 0;
  for (int i = 0; i < q; ++i) rad = std::max(rad, std::abs(z[i]));
  return rad;
}
}  // namespace

double stability_growth(const Model& m, double phi_min, double phi_max) {
  long double worst = 0;
  const int nphi = 5, nk = 129;
  for (int a = 0; a < nphi; ++a) {
    const long double pb = phi_min + (phi_max - phi_min) * (long double)a / (nphi - 1);
    long double w[kMaxQ];
    for (int j = 0; j < m.q; ++j) {   // w_j = d/dphi sum_d G[j][d] phi^d at phi_bar
      long double acc = 0;
      if (m.gF > 0) {
        acc = general_dfeq(m, j, pb);
      } else {
        for (int d = m.D; d >= 1; --d) acc = acc * pb + (long double)d * (long double)m.Gq[j][d];
      }
      w[j] = acc;
    }
    for (int k = 1; k < nk; ++k) {
      const long double kappa = 3.14159265358979323846264L * k / (nk - 1);
      worst = std::max(worst, spectral_radius(m, w, kappa));
    }
  }
  return (double)worst;
}

}  // namespace lbm
