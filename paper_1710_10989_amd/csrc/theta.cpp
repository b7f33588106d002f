// Backward-error thresholds theta_m(u) and the coefficient tables of the product-reduced
// Taylor sequences (host code).
//
// theta_m(u) follows Sec. 1 (eq. eq.theta and the paragraph after it): with
// rho(x) = log(e^{-x} T_m(x)) = sum_{i > m} c_i x^i and f(x) = sum |c_i| x^i cut after 150
// terms, theta is the root of f(theta)/theta = u.  Here the series of g = e^{-x} T_m(x) uses
// the closed form g_i = (-1)^(i+m) C(i-1, m) / i! for i > m (g_0 = 1, g_1..g_m = 0), which
// follows from the alternating partial sum of binomial coefficients; log g comes from the
// power-series recurrence h_n = g_n - (1/n) sum_{k<n} k h_k g_{n-k}; all in long double.
// The root is bracketed by doubling and refined by bisection.
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "expm_internal.h"

namespace expm {
namespace {

typedef long double ld;
constexpr int kTerms = 150;

std::vector<ld> rho_abs(int m) {
  const int K = m + kTerms;
  std::vector<ld> g(K + 1, 0.0L), h(K + 1, 0.0L);
  g[0] = 1.0L;
  for (int i = m + 1; i <= K; ++i) {
    // C(i-1, m) / i!  computed as prod_{t=1..m} (i-m-1+t)/t  /  i!
    ld v = 1.0L;
    for (int t = 1; t <= m; ++t) v *= (ld)(i - m - 1 + t) / (ld)t;
    for (int t = 2; t <= i; ++t) v /= (ld)t;
    g[i] = ((i + m) % 2 == 0) ? v : -v;
  }
  for (int n = 1; n <= K; ++n) {
    ld acc = 0.0L;
    for (int k = m + 1; k <= n - m - 1; ++k) acc += (ld)k * h[k] * g[n - k];
    h[n] = g[n] - acc / (ld)n;
  }
  std::vector<ld> c(kTerms);
  for (int i = 0; i < kTerms; ++i) c[i] = fabsl(h[m + 1 + i]);
  return c;
}

ld bound_over_x(const std::vector<ld> &c, int m, ld x) {
  // f(x)/x = sum_i |c_i| x^(m + i)   (c[i] multiplies x^(m+1+i))
  ld s = 0.0L, p = powl(x, (ld)m);
  for (size_t i = 0; i < c.size(); ++i) {
    s += c[i] * p;
    p *= x;
  }
  return s;
}

std::mutex g_mu;
std::map<std::pair<int, double>, double> g_theta_cache;

}  // namespace

bool theta_of(int m, double u, double *out) {
  bool ok = false;
  for (int i = 0; i < kNumDeg; ++i) ok |= (kDeg[i] == m);
  for (int i = 0; i < kNumPs; ++i) ok |= (kPsDeg[i] == m);
  if (!ok || !(u >= 0x1p-53 && u <= 0x1p-10)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(m, u);
  auto it = g_theta_cache.find(key);
  if (it != g_theta_cache.end()) { *out = it->second; return true; }
  std::vector<ld> c = rho_abs(m);
  ld lo = 0.0L, hi = 1.0L;
  while (bound_over_x(c, m, hi) < (ld)u) { lo = hi; hi *= 2.0L; }
  for (int it2 = 0; it2 < 200; ++it2) {
    ld mid = 0.5L * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (bound_over_x(c, m, mid) < (ld)u) lo = mid; else hi = mid;
  }
  double t = (double)lo;
  if ((ld)t > lo) t = nextafter(t, 0.0);  // round toward zero: the bound must still hold
  g_theta_cache[key] = t;
  *out = t;
  return true;
}

static bool build_consts(double u, Consts *k);

// Consts per u, built once (every call of the library needs them; the thresholds alone take
// thirteen cached lookups).
bool make_consts(double u, Consts *k) {
  static std::mutex mu;
  static std::map<double, Consts> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(u);
    if (it != cache.end()) { *k = it->second; return true; }
  }
  Consts c;
  if (!build_consts(u, &c)) return false;
  std::lock_guard<std::mutex> lk(mu);
  cache.emplace(u, c);
  *k = c;
  return true;
}

static bool build_consts(double u, Consts *k) {
  for (int i = 0; i < kNumDeg; ++i)
    if (!theta_of(kDeg[i], u, &k->theta[i])) return false;
  for (int i = 0; i < kNumPs; ++i)
    if (!theta_of(kPsDeg[i], u, &k->theta_ps[i])) return false;
  // Pade: b_j = (2m - j)! m! / ((2m)! (m - j)! j!) (eq. eq.24), as running products
  auto pade_b = [](int m, double *b) {
    for (int j = 0; j <= m; ++j) {
      ld v = 1.0L;
      for (int t = 0; t < j; ++t) v *= (ld)(m - t) / (ld)(2 * m - t);
      for (int t = 2; t <= j; ++t) v /= (ld)t;
      b[j] = (double)v;
    }
  };
  pade_b(5, k->pade5);
  pade_b(13, k->pade13);
  // theta_10, theta_26 of Table 1, one unit of the third printed digit below the printed value
  // (a printed value may be rounded up; this one is not above the true threshold)
  if (u == 0x1p-53) {
    k->theta_pade[0] = 2.53e-1; k->theta_pade[1] = 5.36;
  } else if (u == 0x1p-24) {
    k->theta_pade[0] = 1.87; k->theta_pade[1] = 11.1;
  } else {
    k->theta_pade[0] = k->theta_pade[1] = 0.0;
  }
  // T_8 (eq. Algorithm83eA), free parameter x3 = 2/3, closed forms in sqrt(177).
  const ld r = sqrtl(177.0L), x3 = 2.0L / 3.0L;
  k->t8[0] = (double)(x3 * (1.0L + r) / 88.0L);                 // x1
  k->t8[1] = (double)((1.0L + r) / 352.0L * x3);                // x2
  k->t8[2] = (double)x3;                                        // x3
  k->t8[3] = (double)((-271.0L + 29.0L * r) / (315.0L * x3));   // x4
  k->t8[4] = (double)(11.0L * (-1.0L + r) / (1260.0L * x3));    // x5
  k->t8[5] = (double)(11.0L * (-9.0L + r) / (5040.0L * x3));    // x6
  k->t8[6] = (double)((89.0L - r) / (5040.0L * x3 * x3));       // x7
  k->t8[7] = 1.0;                                               // y0
  k->t8[8] = 1.0;                                               // y1
  k->t8[9] = (double)((857.0L - 58.0L * r) / 630.0L);           // y2
  // T_12 (eq. poly12): rows B_1..B_4, columns powers I, A, A^2, A^3.
  static const double a12[4][4] = {
      {9.0198e-16, 0.46932117595418237389, -0.20099424927047284052, -0.04623946134063071740},
      {5.31597895759871264183, 1.19926790417132231573, 0.01179296240992997031, 0.01108844528519167989},
      {0.18188869982170434744, 0.05502798439925399070, 0.09351590770535414968, 0.00610700528898058230},
      {-2.0861320e-13, -0.13181061013830184015, -0.02027855540589259079, -0.00675951846863086359}};
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) k->t12[j][i] = a12[j][i];
  // T_18 (eq. poly.18).
  static const double a18[4] = {0.0, -0.100365581030144620, -0.0080292464824115696, -0.0008921384980457299};
  static const double b18[4][5] = {
      {0.0, 0.39784974949964507614, 1.36783778460411719922, 0.49828962252538267755, -0.0006378981945947233},
      {-10.967639605296206259, 1.68015813878906197182, 0.05717798464788655127, -0.0069821012248805208, 0.00003349750170860705},
      {-0.0904316832390810561, -0.0676404519071381907, 0.06759613017704596460, 0.02955525704293155274, -0.0000139180257516060},
      {0.0, 0.0, -0.0923364619367118592, -0.0169364939002081717, -0.0000140086798182036}};
  for (int i = 0; i < 4; ++i) k->t18a[i] = a18[i];
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 5; ++i) k->t18b[j][i] = b18[j][i];
  return true;
}

}  // namespace expm
