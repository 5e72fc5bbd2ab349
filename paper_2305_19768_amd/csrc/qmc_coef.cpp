// qmc_coef.cpp -- coefficients of weighted sums given as expressions (Sec. 2.4).
//
// A coefficient is an arithmetic expression in the dimensional regulator and in
// kinematic symbols.  It is evaluated with the symbols replaced by the caller's values
// and expanded into a Laurent series in the regulator, in exact rational arithmetic
// (no precision is lost to cancellations in large reduction coefficients); the series
// coefficients are then rounded to the nearest double.  Host code only.
//
// Arithmetic: arbitrary-precision integers (32-bit limbs, schoolbook products, long
// division after Knuth, Euclid's gcd), rationals in lowest terms, complex rationals
// (the imaginary unit is the symbol I).  Series: truncated Laurent series with tracked
// precision -- a series knows its coefficients for every order below `prec`; products,
// inverses and powers propagate `prec` exactly (an inverse of a series with leading order
// a and precision P is known below P - 2a), and every series is cut at a working order
// H.  If the result is not known far enough, the evaluation is repeated with a larger H.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "qmc_plan.h"

namespace {

struct CoefError : std::runtime_error {
  explicit CoefError(const std::string &m) : std::runtime_error(m) {}
};
// thrown when the working order H was too small to decide a division
struct NeedMoreOrders {};

constexpr size_t kMaxLimbs = 1 << 16;   // 2^21 bits per integer
constexpr int kMaxDepth = 2000;         // nesting of the expression
constexpr int64_t kInf = int64_t(1) << 40;

// ------------------------------------------------------------ natural numbers
using Nat = std::vector<uint32_t>;   // little-endian limbs, no leading zero limb

void trim(Nat &a) {
  while (!a.empty() && a.back() == 0) a.pop_back();
}

void check_size(const Nat &a) {
  if (a.size() > kMaxLimbs) throw CoefError("integer too large in the exact evaluation");
}

int cmp(const Nat &a, const Nat &b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

Nat add(const Nat &a, const Nat &b) {
  const Nat &x = a.size() >= b.size() ? a : b, &y = a.size() >= b.size() ? b : a;
  Nat r(x.size() + 1);
  uint64_t c = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    const uint64_t s = (uint64_t)x[i] + (i < y.size() ? y[i] : 0) + c;
    r[i] = (uint32_t)s;
    c = s >> 32;
  }
  r[x.size()] = (uint32_t)c;
  trim(r);
  check_size(r);
  return r;
}

// a - b for a >= b
Nat sub(const Nat &a, const Nat &b) {
  Nat r(a.size());
  int64_t br = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    int64_t t = (int64_t)a[i] - (i < b.size() ? (int64_t)b[i] : 0) - br;
    br = t < 0;
    r[i] = (uint32_t)(t + (br << 32));
  }
  trim(r);
  return r;
}

Nat mul(const Nat &a, const Nat &b) {
  if (a.empty() || b.empty()) return {};
  if (a.size() + b.size() > kMaxLimbs) throw CoefError("integer too large in the exact evaluation");
  Nat r(a.size() + b.size(), 0);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t c = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      const uint64_t t = (uint64_t)a[i] * b[j] + r[i + j] + c;
      r[i + j] = (uint32_t)t;
      c = t >> 32;
    }
    r[i + b.size()] = (uint32_t)c;
  }
  trim(r);
  return r;
}

Nat mul_small(const Nat &a, uint32_t m, uint32_t add_in = 0) {
  Nat r(a.size() + 1);
  uint64_t c = add_in;
  for (size_t i = 0; i < a.size(); ++i) {
    const uint64_t t = (uint64_t)a[i] * m + c;
    r[i] = (uint32_t)t;
    c = t >> 32;
  }
  r[a.size()] = (uint32_t)c;
  trim(r);
  check_size(r);
  return r;
}

int64_t bitlen(const Nat &a) {
  if (a.empty()) return 0;
  return 32 * (int64_t)(a.size() - 1) + (32 - __builtin_clz(a.back()));
}

Nat shl(const Nat &a, int64_t s) {
  if (a.empty()) return {};
  const size_t w = (size_t)(s / 32);
  const int b = (int)(s % 32);
  if (a.size() + w + 1 > kMaxLimbs) throw CoefError("integer too large in the exact evaluation");
  Nat r(a.size() + w + 1, 0);
  for (size_t i = 0; i < a.size(); ++i) {
    r[i + w] |= a[i] << b;
    if (b) r[i + w + 1] |= (uint32_t)((uint64_t)a[i] >> (32 - b));
  }
  trim(r);
  return r;
}

Nat shr(const Nat &a, int64_t s) {
  const size_t w = (size_t)(s / 32);
  const int b = (int)(s % 32);
  if (w >= a.size()) return {};
  Nat r(a.size() - w, 0);
  for (size_t i = 0; i < r.size(); ++i) {
    uint64_t v = a[i + w] >> b;
    if (b && i + w + 1 < a.size()) v |= (uint64_t)a[i + w + 1] << (32 - b);
    r[i] = (uint32_t)v;
  }
  trim(r);
  return r;
}

// q = u / v, r = u mod v (v != 0): long division with normalised divisor and
// two-limb quotient estimates, corrected by at most two decrements and an add-back.
void divmod(const Nat &u_in, const Nat &v_in, Nat &q, Nat &r) {
  if (v_in.empty()) throw CoefError("division by zero");
  if (cmp(u_in, v_in) < 0) {
    q.clear();
    r = u_in;
    return;
  }
  if (v_in.size() == 1) {
    const uint64_t dv = v_in[0];
    q.assign(u_in.size(), 0);
    uint64_t rem = 0;
    for (size_t i = u_in.size(); i-- > 0;) {
      const uint64_t cur = (rem << 32) | u_in[i];
      q[i] = (uint32_t)(cur / dv);
      rem = cur % dv;
    }
    trim(q);
    r.clear();
    if (rem) r.push_back((uint32_t)rem);
    return;
  }
  const int s = __builtin_clz(v_in.back());
  Nat v = shl(v_in, s);
  Nat u = shl(u_in, s);
  u.resize(u_in.size() + 1, 0);
  const size_t n = v.size(), m = u_in.size() - n;
  q.assign(m + 1, 0);
  const uint64_t B = uint64_t(1) << 32;
  for (size_t j = m + 1; j-- > 0;) {
    const uint64_t num = ((uint64_t)u[j + n] << 32) | u[j + n - 1];
    uint64_t qhat = num / v[n - 1], rhat = num % v[n - 1];
    while (qhat >= B || qhat * v[n - 2] > ((rhat << 32) | u[j + n - 2])) {
      --qhat;
      rhat += v[n - 1];
      if (rhat >= B) break;
    }
    int64_t borrow = 0;
    uint64_t carry = 0;
    for (size_t i = 0; i < n; ++i) {
      const uint64_t p = qhat * v[i] + carry;
      carry = p >> 32;
      const int64_t t = (int64_t)u[i + j] - (int64_t)(p & 0xffffffffu) - borrow;
      u[i + j] = (uint32_t)t;
      borrow = t < 0;
    }
    const int64_t t = (int64_t)u[j + n] - (int64_t)carry - borrow;
    u[j + n] = (uint32_t)t;
    if (t < 0) {   // the estimate was one too large: add the divisor back
      --qhat;
      uint64_t c = 0;
      for (size_t i = 0; i < n; ++i) {
        const uint64_t sm = (uint64_t)u[i + j] + v[i] + c;
        u[i + j] = (uint32_t)sm;
        c = sm >> 32;
      }
      u[j + n] += (uint32_t)c;
    }
    q[j] = (uint32_t)qhat;
  }
  trim(q);
  u.resize(n);
  trim(u);
  r = shr(u, s);
}

Nat gcd(Nat a, Nat b) {
  while (!b.empty()) {
    Nat q, r;
    divmod(a, b, q, r);
    a = std::move(b);
    b = std::move(r);
  }
  return a;
}

Nat nat_from(uint64_t v) {
  Nat r;
  while (v) {
    r.push_back((uint32_t)v);
    v >>= 32;
  }
  return r;
}

// ------------------------------------------------------------------ rationals
struct Q {
  bool neg = false;
  Nat num;           // |numerator|; empty for zero
  Nat den{1};        // > 0
  bool zero() const { return num.empty(); }
};

Q normalize(bool neg, Nat num, Nat den) {
  if (den.empty()) throw CoefError("division by zero");
  Q r;
  if (num.empty()) return r;
  Nat g = gcd(num, den);
  if (!(g.size() == 1 && g[0] == 1)) {
    Nat t;
    divmod(num, g, r.num, t);
    divmod(den, g, r.den, t);
  } else {
    r.num = std::move(num);
    r.den = std::move(den);
  }
  r.neg = neg;
  return r;
}

Q q_neg(Q a) {
  if (!a.zero()) a.neg = !a.neg;
  return a;
}

Q q_add(const Q &a, const Q &b) {
  if (a.zero()) return b;
  if (b.zero()) return a;
  const Nat x = mul(a.num, b.den), y = mul(b.num, a.den);
  Nat den = mul(a.den, b.den);
  if (a.neg == b.neg) return normalize(a.neg, add(x, y), std::move(den));
  const int c = cmp(x, y);
  if (c == 0) return Q{};
  return c > 0 ? normalize(a.neg, sub(x, y), std::move(den)) : normalize(b.neg, sub(y, x), std::move(den));
}

Q q_mul(const Q &a, const Q &b) {
  if (a.zero() || b.zero()) return Q{};
  return normalize(a.neg != b.neg, mul(a.num, b.num), mul(a.den, b.den));
}

Q q_inv(const Q &a) {
  if (a.zero()) throw CoefError("division by zero");
  return normalize(a.neg, a.den, a.num);
}

Q q_int(int64_t v) {
  Q r;
  if (v == 0) return r;
  r.neg = v < 0;
  r.num = nat_from(v < 0 ? (uint64_t)(-(v + 1)) + 1 : (uint64_t)v);
  return r;
}

// nearest double (ties to even), with gradual underflow; overflow is an error
double q_to_double(const Q &a) {
  if (a.zero()) return 0.0;
  const int64_t la = bitlen(a.num), lb = bitlen(a.den);
  const int64_t s = 66 - (la - lb);          // quotient with 65..67 bits
  Nat A = s >= 0 ? shl(a.num, s) : a.num, Bd = s >= 0 ? a.den : shl(a.den, -s);
  Nat qt, rm;
  divmod(A, Bd, qt, rm);
  const bool sticky = !rm.empty();
  const int64_t qb = bitlen(qt);
  const int64_t E = qb - 1 - s;               // value in [2^E, 2^(E+1))
  if (E > 1023) throw CoefError("coefficient outside the double range");
  if (E < -1075) return a.neg ? -0.0 : 0.0;   // below half the smallest subnormal
  int64_t keep = 53;
  if (E < -1022) keep = std::max<int64_t>(0, 53 - (-1022 - E));
  const int64_t drop = qb - keep;             // >= 12
  Nat M = shr(qt, drop);
  uint64_t mant = 0;
  for (size_t i = 0; i < M.size() && i < 2; ++i) mant |= (uint64_t)M[i] << (32 * i);
  // the dropped bits against half an ulp
  const Nat low = sub(qt, shl(M, drop));
  const Nat half = shl(Nat{1}, drop - 1);
  const int c = cmp(low, half);
  if (c > 0 || (c == 0 && (sticky || (mant & 1)))) ++mant;
  const double v = std::ldexp((double)mant, (int)(drop - s));
  if (!std::isfinite(v)) throw CoefError("coefficient outside the double range");
  return a.neg ? -v : v;
}

// exact decimal literal: digits [. digits] [e|E [+|-] digits]
Q q_decimal(const std::string &t) {
  Nat mant;
  int64_t exp10 = 0;
  size_t i = 0;
  bool any = false;
  for (; i < t.size() && isdigit((unsigned char)t[i]); ++i, any = true)
    mant = mul_small(mant, 10, (uint32_t)(t[i] - '0'));
  if (i < t.size() && t[i] == '.') {
    for (++i; i < t.size() && isdigit((unsigned char)t[i]); ++i, any = true) {
      mant = mul_small(mant, 10, (uint32_t)(t[i] - '0'));
      --exp10;
    }
  }
  if (!any) throw CoefError("malformed number '" + t + "'");
  if (i < t.size() && (t[i] == 'e' || t[i] == 'E')) {
    ++i;
    bool eneg = false;
    if (i < t.size() && (t[i] == '+' || t[i] == '-')) eneg = t[i++] == '-';
    int64_t e = 0;
    bool digits = false;
    for (; i < t.size() && isdigit((unsigned char)t[i]); ++i, digits = true) {
      e = e * 10 + (t[i] - '0');
      if (e > 100000) throw CoefError("exponent too large in '" + t + "'");
    }
    if (!digits) throw CoefError("malformed number '" + t + "'");
    exp10 += eneg ? -e : e;
  }
  if (i != t.size()) throw CoefError("malformed number '" + t + "'");
  Nat p10{1};
  for (int64_t k = 0; k < (exp10 < 0 ? -exp10 : exp10); ++k) p10 = mul_small(p10, 10);
  return exp10 >= 0 ? normalize(false, mul(mant, p10), Nat{1}) : normalize(false, mant, p10);
}

// ---------------------------------------------------------- complex rationals
struct C {
  Q re, im;
  bool zero() const { return re.zero() && im.zero(); }
};

C c_add(const C &a, const C &b) { return C{q_add(a.re, b.re), q_add(a.im, b.im)}; }
C c_neg(const C &a) { return C{q_neg(a.re), q_neg(a.im)}; }
C c_mul(const C &a, const C &b) {
  if (a.im.zero() && b.im.zero()) return C{q_mul(a.re, b.re), Q{}};
  return C{q_add(q_mul(a.re, b.re), q_neg(q_mul(a.im, b.im))),
           q_add(q_mul(a.re, b.im), q_mul(a.im, b.re))};
}
C c_inv(const C &a) {
  if (a.zero()) throw CoefError("division by zero");
  if (a.im.zero()) return C{q_inv(a.re), Q{}};
  const Q n2 = q_add(q_mul(a.re, a.re), q_mul(a.im, a.im));
  const Q r = q_inv(n2);
  return C{q_mul(a.re, r), q_neg(q_mul(a.im, r))};
}

// -------------------------------------------------------------------- series
struct Ser {
  int64_t lo = 0;        // order of c[0]
  int64_t prec = kInf;   // coefficients known for every order < prec
  std::vector<C> c;      // orders lo .. lo + c.size() - 1; known orders beyond are zero
};

int64_t sat_add(int64_t a, int64_t b) {
  if (a >= kInf || b >= kInf) return kInf;
  return a + b;
}

// Cut a series at the working order H: terms at orders >= H are dropped, and if a
// non-zero one was, the series is known only below H.  Leading and trailing zero terms
// are removed (orders between the last term and prec are known to be zero).
void tidy(Ser &a, int64_t H) {
  size_t keep = 0;
  while (keep < a.c.size() && a.lo + (int64_t)keep < a.prec && a.lo + (int64_t)keep < H) ++keep;
  bool dropped = false;
  for (size_t i = keep; i < a.c.size(); ++i)
    if (a.lo + (int64_t)i < a.prec && !a.c[i].zero()) dropped = true;
  a.c.resize(keep);
  if (dropped) a.prec = std::min(a.prec, H);
  size_t z = 0;
  while (z < a.c.size() && a.c[z].zero()) ++z;
  if (z) {
    a.c.erase(a.c.begin(), a.c.begin() + (std::ptrdiff_t)z);
    a.lo += (int64_t)z;
  }
  while (!a.c.empty() && a.c.back().zero()) a.c.pop_back();
  if (a.c.empty()) a.lo = 0;
}

// lowest order that may be non-zero
int64_t lead(const Ser &a) { return a.c.empty() ? a.prec : a.lo; }

bool exact_zero(const Ser &a) { return a.c.empty() && a.prec >= kInf; }

Ser s_const(const C &v) {
  Ser r;
  if (!v.zero()) r.c.push_back(v);
  return r;
}

Ser s_add(const Ser &a, const Ser &b, int64_t H) {
  if (exact_zero(a)) return b;
  if (exact_zero(b)) return a;
  Ser r;
  r.prec = std::min(a.prec, b.prec);
  if (a.c.empty() && b.c.empty()) return r;
  const int64_t lo = a.c.empty() ? b.lo : b.c.empty() ? a.lo : std::min(a.lo, b.lo);
  const int64_t hi = std::max(a.lo + (int64_t)a.c.size(), b.lo + (int64_t)b.c.size());
  r.lo = lo;
  for (int64_t o = lo; o < hi && o < r.prec; ++o) {
    C v;
    if (o >= a.lo && o < a.lo + (int64_t)a.c.size()) v = a.c[(size_t)(o - a.lo)];
    if (o >= b.lo && o < b.lo + (int64_t)b.c.size()) v = c_add(v, b.c[(size_t)(o - b.lo)]);
    r.c.push_back(v);
  }
  tidy(r, H);
  return r;
}

Ser s_neg(Ser a) {
  for (C &v : a.c) v = c_neg(v);
  return a;
}

Ser s_mul(const Ser &a, const Ser &b, int64_t H) {
  if (exact_zero(a) || exact_zero(b)) return Ser{};
  Ser r;
  r.prec = std::min(sat_add(a.prec, lead(b)), sat_add(b.prec, lead(a)));
  if (a.c.empty() || b.c.empty()) return r;
  r.lo = a.lo + b.lo;
  const int64_t full = (int64_t)(a.c.size() + b.c.size()) - 1;
  // terms at orders >= H are not formed; if any could be non-zero, prec drops to H
  if (r.lo + full > H) r.prec = std::min(r.prec, H);
  const int64_t n = std::min(full, r.prec - r.lo);
  if (n <= 0) {
    r.lo = 0;
    return r;
  }
  r.c.assign((size_t)n, C{});
  for (size_t i = 0; i < a.c.size() && (int64_t)i < n; ++i)
    for (size_t j = 0; j < b.c.size() && (int64_t)(i + j) < n; ++j)
      r.c[i + j] = c_add(r.c[i + j], c_mul(a.c[i], b.c[j]));
  tidy(r, H);
  return r;
}

// 1/a: a = eps^lo (c0 + c1 eps + ...) known below prec gives
// eps^-lo (b0 + b1 eps + ...) with b0 = 1/c0, b_k = -b0 sum_{j=1..k} c_j b_{k-j}, known
// below prec - 2 lo.  An exact single term inverts exactly.
Ser s_inv(const Ser &a, int64_t H) {
  if (a.c.empty()) {
    if (a.prec >= kInf) throw CoefError("division by zero");
    throw NeedMoreOrders{};   // zero as far as known: the divisor needs more orders
  }
  Ser r;
  r.lo = -a.lo;
  const C b0 = c_inv(a.c[0]);
  if (a.c.size() == 1 && a.prec >= kInf) {
    r.c.push_back(b0);
    tidy(r, H);
    return r;
  }
  r.prec = std::min(a.prec >= kInf ? kInf : a.prec - 2 * a.lo, H);
  const int64_t n = r.prec - r.lo;
  if (n <= 0) {
    r.lo = 0;
    return r;
  }
  r.c.reserve((size_t)n);
  r.c.push_back(b0);
  for (int64_t k = 1; k < n; ++k) {
    C acc;
    for (int64_t j = 1; j <= k && j < (int64_t)a.c.size(); ++j)
      acc = c_add(acc, c_mul(a.c[(size_t)j], r.c[(size_t)(k - j)]));
    r.c.push_back(c_neg(c_mul(b0, acc)));
  }
  tidy(r, H);
  return r;
}

Ser s_pow(Ser a, int64_t e, int64_t H) {
  if (e < 0) {
    a = s_inv(a, H);
    e = -e;
  }
  Ser r = s_const(C{q_int(1), Q{}});
  while (e) {
    if (e & 1) r = s_mul(r, a, H);
    e >>= 1;
    if (e) a = s_mul(a, a, H);
  }
  return r;
}

// ------------------------------------------------------------------ parsing
struct Node {
  enum Kind { NUM, SYM, EPS, IMAG, NEG, ADD, SUB, MUL, DIV, POW } kind;
  Q num;
  std::string name;
  std::unique_ptr<Node> a, b;
};
using P = std::unique_ptr<Node>;

P mk(Node::Kind k, P a = nullptr, P b = nullptr) {
  P n(new Node{k, Q{}, std::string(), nullptr, nullptr});
  n->a = std::move(a);
  n->b = std::move(b);
  return n;
}

struct Parser {
  const std::string &s;
  const std::string &reg;
  size_t i = 0;
  int depth = 0;

  void ws() {
    while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  }
  bool eat(const char *t) {
    ws();
    const size_t n = strlen(t);
    if (s.compare(i, n, t) == 0) {
      i += n;
      return true;
    }
    return false;
  }
  [[noreturn]] void err(const std::string &m) {
    throw CoefError(m + " at position " + std::to_string(i) + " of '" +
                    (s.size() > 60 ? s.substr(0, 60) + "..." : s) + "'");
  }
  P expr() {
    if (++depth > kMaxDepth) err("expression nested too deeply");
    P l = term();
    for (;;) {
      if (eat("+")) l = mk(Node::ADD, std::move(l), term());
      else if (eat("-")) l = mk(Node::SUB, std::move(l), term());
      else break;
    }
    --depth;
    return l;
  }
  P term() {
    P l = unary();
    for (;;) {
      ws();
      if (i + 1 < s.size() && s[i] == '*' && s[i + 1] == '*') break;   // power
      if (eat("*")) l = mk(Node::MUL, std::move(l), unary());
      else if (eat("/")) l = mk(Node::DIV, std::move(l), unary());
      else break;
    }
    return l;
  }
  P unary() {
    if (++depth > kMaxDepth) err("expression nested too deeply");
    P r;
    if (eat("-")) r = mk(Node::NEG, unary());
    else if (eat("+")) r = unary();
    else r = power();
    --depth;
    return r;
  }
  P power() {
    P base = primary();
    if (eat("^") || eat("**")) return mk(Node::POW, std::move(base), unary());   // right-assoc
    return base;
  }
  P primary() {
    ws();
    if (i >= s.size()) err("unexpected end");
    if (eat("(")) {
      P e = expr();
      if (!eat(")")) err("missing ')'");
      return e;
    }
    const char c = s[i];
    if (isdigit((unsigned char)c) || c == '.') {
      const size_t b = i;
      while (i < s.size() && (isdigit((unsigned char)s[i]) || s[i] == '.')) ++i;
      if (i < s.size() && (s[i] == 'e' || s[i] == 'E')) {
        size_t k = i + 1;
        if (k < s.size() && (s[k] == '+' || s[k] == '-')) ++k;
        if (k < s.size() && isdigit((unsigned char)s[k])) {
          i = k;
          while (i < s.size() && isdigit((unsigned char)s[i])) ++i;
        }
      }
      P n = mk(Node::NUM);
      n->num = q_decimal(s.substr(b, i - b));
      return n;
    }
    if (isalpha((unsigned char)c) || c == '_') {
      const size_t b = i;
      while (i < s.size() && (isalnum((unsigned char)s[i]) || s[i] == '_')) ++i;
      const std::string name = s.substr(b, i - b);
      ws();
      if (i < s.size() && s[i] == '(') err("functions are not supported ('" + name + "')");
      if (name == reg) return mk(Node::EPS);
      if (name == "I") return mk(Node::IMAG);
      P n = mk(Node::SYM);
      n->name = name;
      return n;
    }
    err(std::string("unexpected character '") + c + "'");
  }
};

P parse(const std::string &s, const std::string &reg) {
  Parser p{s, reg};
  P e = p.expr();
  p.ws();
  if (p.i != s.size()) p.err("unexpected trailing input");
  return e;
}

// Symbol values are expressions themselves (they may depend on the regulator, e.g. a
// dimension 4 - 2 eps); a value may use only symbols defined before it.
struct Env {
  std::map<std::string, P> values;
};

void check_symbols(const Node &x, const Env &env) {
  if (x.kind == Node::SYM && !env.values.count(x.name))
    throw CoefError("no value given for symbol '" + x.name + "'");
  if (x.a) check_symbols(*x.a, env);
  if (x.b) check_symbols(*x.b, env);
}

C eval_const(const Node &n, const Env &env);

Ser eval(const Node &n, const Env &env, int64_t H) {
  switch (n.kind) {
    case Node::NUM: {
      Ser r = s_const(C{n.num, Q{}});
      tidy(r, H);
      return r;
    }
    case Node::IMAG: {
      Ser r = s_const(C{Q{}, q_int(1)});
      tidy(r, H);
      return r;
    }
    case Node::EPS: {
      Ser r;
      r.lo = 1;
      r.c.push_back(C{q_int(1), Q{}});
      tidy(r, H);
      return r;
    }
    case Node::SYM: {
      auto it = env.values.find(n.name);
      if (it == env.values.end()) throw CoefError("no value given for symbol '" + n.name + "'");
      return eval(*it->second, env, H);
    }
    case Node::NEG: return s_neg(eval(*n.a, env, H));
    case Node::ADD: return s_add(eval(*n.a, env, H), eval(*n.b, env, H), H);
    case Node::SUB: return s_add(eval(*n.a, env, H), s_neg(eval(*n.b, env, H)), H);
    case Node::MUL: return s_mul(eval(*n.a, env, H), eval(*n.b, env, H), H);
    case Node::DIV: return s_mul(eval(*n.a, env, H), s_inv(eval(*n.b, env, H), H), H);
    case Node::POW: {
      const C e = eval_const(*n.b, env);
      if (!e.im.zero() || !(e.re.den.size() == 1 && e.re.den[0] == 1) || e.re.num.size() > 1)
        throw CoefError("exponents must be integers (a power with a non-integer or "
                        "regulator-dependent exponent is not a rational function)");
      const int64_t m = e.re.num.empty() ? 0 : (int64_t)e.re.num[0];
      if (m > 100000) throw CoefError("exponent too large");
      return s_pow(eval(*n.a, env, H), e.re.neg ? -m : m, H);
    }
  }
  throw CoefError("bad expression");
}

// value of a regulator-free sub-expression (exponents, symbol values)
bool has_regulator(const Node &x, const Env &env) {
  if (x.kind == Node::EPS) return true;
  if (x.kind == Node::SYM) {
    auto it = env.values.find(x.name);
    return it != env.values.end() && has_regulator(*it->second, env);
  }
  return (x.a && has_regulator(*x.a, env)) || (x.b && has_regulator(*x.b, env));
}

C eval_const(const Node &n, const Env &env) {
  if (has_regulator(n, env))
    throw CoefError("exponents must not depend on the regulator");
  Ser r = eval(n, env, 1);
  for (size_t j = 0; j < r.c.size(); ++j)
    if (r.lo + (int64_t)j == 0) return r.c[j];
  return C{};
}

// Series of `expr` known at least below order `need` (exclusive); also returns the
// exact leading order when the series is not identically zero.
Ser expand(const Node &root, const Env &env, int64_t need) {
  int64_t H = need + 4;
  for (int attempt = 0; attempt < 64; ++attempt) {
    try {
      Ser r = eval(root, env, H);
      if (r.prec >= need) return r;
      H += std::max<int64_t>(need - r.prec, 1) + 2;
    } catch (const NeedMoreOrders &) {
      H += 4 + attempt * 4;
    }
  }
  throw CoefError("expansion did not reach the requested order (cancellation beyond the "
                  "working depth)");
}

}  // namespace

extern "C" qmc_status qmc_coef_series(const char *expr, const char *regulator, int32_t n_symbols,
                                      const char *const *names, const char *const *values,
                                      int32_t order_lo, int32_t n_terms, int32_t *leading_order,
                                      double *re, double *im) {
  qmc::g_last_error.clear();
  if (!expr || !regulator || (n_symbols > 0 && (!names || !values)) || n_symbols < 0 ||
      n_terms < 0 || (n_terms > 0 && (!re || !im)))
    return qmc::fail(QMC_E_INVAL, "NULL argument or negative count");
  if (n_terms > 4096) return qmc::fail(QMC_E_INVAL, "n_terms = %d above 4096", n_terms);
  if (order_lo < -100000 || order_lo > 100000)
    return qmc::fail(QMC_E_INVAL, "order_lo = %d outside [-1e5, 1e5]", order_lo);
  try {
    const std::string reg(regulator), src(expr);
    if (reg.empty() || reg == "I") throw CoefError("the regulator needs a name other than I");
    Env env;
    for (int32_t k = 0; k < n_symbols; ++k) {
      if (!names[k] || !values[k]) throw CoefError("NULL symbol name or value");
      const std::string nm(names[k]);
      if (nm == reg || nm == "I") throw CoefError("symbol '" + nm + "' is reserved");
      if (env.values.count(nm)) throw CoefError("symbol '" + nm + "' given twice");
      P v = parse(values[k], reg);
      check_symbols(*v, env);
      env.values[nm] = std::move(v);
    }
    P root = parse(src, reg);
    check_symbols(*root, env);
    // leading order: expand until a non-zero term is known (or the series is exactly 0)
    int64_t need = (int64_t)order_lo + n_terms;
    Ser r = expand(*root, env, need);
    int64_t lead_o = r.c.empty() ? kInf : r.lo;
    for (int extra = 0; r.c.empty() && r.prec < kInf && extra < 64; ++extra) {
      need = r.prec + 8;
      r = expand(*root, env, need);
      lead_o = r.c.empty() ? kInf : r.lo;
    }
    if (r.c.empty() && r.prec < kInf)
      throw CoefError("could not determine the leading order (zero to high order)");
    if (leading_order) leading_order[0] = lead_o >= kInf ? INT32_MAX : (int32_t)lead_o;
    if (n_terms > 0) {
      if (lead_o < order_lo)
        return qmc::fail(QMC_E_INVAL, "coefficient has a term at order %lld below order_lo = %d",
                         (long long)lead_o, order_lo);
      for (int32_t j = 0; j < n_terms; ++j) {
        const int64_t o = (int64_t)order_lo + j;
        C v;
        if (!r.c.empty() && o >= r.lo && o < r.lo + (int64_t)r.c.size()) v = r.c[o - r.lo];
        re[j] = q_to_double(v.re);
        im[j] = q_to_double(v.im);
      }
    }
    return QMC_OK;
  } catch (const CoefError &e) {
    return qmc::fail(QMC_E_INVAL, "%s", e.what());
  } catch (const std::bad_alloc &) {
    return qmc::fail(QMC_E_NOMEM, "out of host memory in the exact evaluation");
  }
}
