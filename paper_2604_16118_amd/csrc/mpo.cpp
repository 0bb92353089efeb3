// Host construction of the block-sparse MPO (see mpo.hpp for the scheme).
#include "mpo.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <unordered_map>

namespace pv {
namespace {

enum : uint8_t { OP_CRE = 0, OP_ANN = 1 };

struct Term {
  double c;
  uint8_t n;        // number of operators (2 or 4)
  uint8_t type[4];  // OP_CRE / OP_ANN in product order
  uint8_t pos[4];   // orbital (0-based)
};

// 2x2 local matrices, row = output occupation, column = input occupation.
using M2 = std::array<double, 4>;  // {m00, m01, m10, m11}
constexpr M2 kI = {1, 0, 0, 1};
constexpr M2 kS = {1, 0, 0, -1};
constexpr M2 kA = {0, 1, 0, 0};   // annihilation: |0><1|
constexpr M2 kAt = {0, 0, 1, 0};  // creation: |1><0|

inline M2 mul(const M2& a, const M2& b) {
  return {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
          a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
}

enum : uint64_t { TAG_I = 0, TAG_F = 1, TAG_L = 2, TAG_R = 3 };

// Key of a term's bond state at cut m (slots with pos < m are left of the cut).
inline uint64_t key_at(const Term& t, int m, int L) {
  int nl = 0;
  for (int s = 0; s < t.n; ++s) nl += t.pos[s] < m;
  const int nr = t.n - nl;
  if (nl == 0) return TAG_I;
  if (nr == 0) return TAG_F;
  const bool left = nl < nr || (nl == nr && 2 * m < L);
  uint64_t key = left ? TAG_L : TAG_R;
  int cnt = 0;
  for (int s = 0; s < t.n; ++s) {
    const bool is_left = t.pos[s] < m;
    if (is_left == left) {
      key |= uint64_t((t.type[s] << 7) | t.pos[s]) << (8 + 8 * cnt);
      ++cnt;
    }
  }
  key |= uint64_t(cnt) << 2;
  return key;
}

inline int key_charge(uint64_t key) {
  const uint64_t tag = key & 3;
  if (tag == TAG_I || tag == TAG_F) return 0;
  const int cnt = int((key >> 2) & 7);
  int q = 0;
  for (int s = 0; s < cnt; ++s) {
    const int ty = int((key >> (8 + 8 * s + 7)) & 1);
    q += ty == OP_CRE ? 1 : -1;
  }
  return tag == TAG_L ? q : -q;
}

// Sign relating the exact left factor of a left-keyed term to the canonical operator of
// its key: moving each parity string (from a slot right of the cut) to the end passes
// every left slot that follows it in product order.
inline double left_sign(const Term& t, int m) {
  int swaps = 0;
  for (int s = 0; s < t.n; ++s) {
    if (t.pos[s] >= m) {
      for (int u = s + 1; u < t.n; ++u) swaps += t.pos[u] < m;
    }
  }
  return (swaps & 1) ? -1.0 : 1.0;
}

// Factor of the term on site m: ordered product of the per-slot factors.
inline M2 site_factor(const Term& t, int m) {
  M2 f = kI;
  for (int s = 0; s < t.n; ++s) {
    const M2& g = t.pos[s] < m ? kI : (t.pos[s] == m ? (t.type[s] == OP_CRE ? kAt : kA) : kS);
    f = mul(f, g);
  }
  return f;
}

struct CutStates {
  std::unordered_map<uint64_t, int> id;
  std::vector<uint64_t> keys;
};

}  // namespace

Mpo build_mpo(int L, const double* h, const double* v, double diag_shift) {
  if (L < 1 || L > 127) throw std::runtime_error("build_mpo: L out of range [1,127]");
  std::vector<Term> terms;
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      const double c = h[i * L + j] + (i == j ? diag_shift : 0.0);
      if (c == 0.0) continue;
      terms.push_back(Term{c, 2, {OP_CRE, OP_ANN, 0, 0}, {uint8_t(i), uint8_t(j), 0, 0}});
    }
  auto V = [&](int i, int j, int k, int l) { return v[((size_t(i) * L + j) * L + k) * L + l]; };
  for (int i = 0; i < L; ++i)
    for (int j = i + 1; j < L; ++j)
      for (int k = 0; k < L; ++k)
        for (int l = k + 1; l < L; ++l) {
          const double c = V(i, j, k, l) - V(j, i, k, l) - V(i, j, l, k) + V(j, i, l, k);
          if (c == 0.0) continue;
          terms.push_back(Term{c, 4, {OP_CRE, OP_CRE, OP_ANN, OP_ANN},
                               {uint8_t(i), uint8_t(j), uint8_t(k), uint8_t(l)}});
        }
  for (const Term& t : terms)
    if (!std::isfinite(t.c)) throw std::runtime_error("build_mpo: non-finite integral");

  Mpo mpo;
  mpo.L = L;
  mpo.n_terms = int64_t(terms.size());
  std::vector<CutStates> cuts(L + 1);
  // states of every cut, ordered by (charge, key)
#pragma omp parallel for schedule(dynamic)
  for (int m = 0; m <= L; ++m) {
    std::unordered_map<uint64_t, int> seen;
    for (const Term& t : terms) seen.emplace(key_at(t, m, L), 0);
    if (m == 0 || m == L) seen.emplace(m == 0 ? uint64_t(TAG_I) : uint64_t(TAG_F), 0);
    std::vector<uint64_t> keys;
    keys.reserve(seen.size());
    for (auto& kv : seen) keys.push_back(kv.first);
    std::sort(keys.begin(), keys.end(), [](uint64_t a, uint64_t b) {
      const int qa = key_charge(a), qb = key_charge(b);
      return qa != qb ? qa < qb : a < b;
    });
    CutStates cs;
    cs.keys = keys;
    for (size_t b = 0; b < keys.size(); ++b) cs.id.emplace(keys[b], int(b));
    cuts[m] = std::move(cs);
  }
  mpo.w.resize(L + 1);
  mpo.charge.resize(L + 1);
  mpo.qoff.resize(L + 1);
  for (int m = 0; m <= L; ++m) {
    const auto& keys = cuts[m].keys;
    mpo.w[m] = int(keys.size());
    mpo.charge[m].resize(keys.size());
    std::array<int, 6> off{};
    for (size_t b = 0; b < keys.size(); ++b) {
      const int q = key_charge(keys[b]);
      if (q < -2 || q > 2) throw std::runtime_error("build_mpo: bond charge out of range");
      mpo.charge[m][b] = int8_t(q);
    }
    for (int q = -2; q <= 2; ++q) {
      off[q + 3] = off[q + 2];
      for (size_t b = 0; b < keys.size(); ++b) off[q + 3] += mpo.charge[m][b] == q;
    }
    mpo.qoff[m] = off;
  }
  if (mpo.w[0] != 1 || mpo.w[L] != 1) throw std::runtime_error("build_mpo: boundary bond is not 1");

  mpo.site.resize(L);
  std::vector<std::string> errors(L);
#pragma omp parallel for schedule(dynamic)
  for (int m = 0; m < L; ++m) {
    struct Entry { M2 f; bool set_once; };
    std::unordered_map<uint64_t, Entry> ent;
    const auto& id0 = cuts[m].id;
    const auto& id1 = cuts[m + 1].id;
    for (const Term& t : terms) {
      const uint64_t k0 = key_at(t, m, L), k1 = key_at(t, m + 1, L);
      const int b = id0.at(k0), bp = id1.at(k1);
      const uint64_t tag0 = k0 & 3, tag1 = k1 & 3;
      const bool left0 = tag0 == TAG_I || tag0 == TAG_L;
      const bool left1 = tag1 == TAG_I || tag1 == TAG_L;
      const M2 f = site_factor(t, m);
      const uint64_t pk = (uint64_t(uint32_t(b)) << 32) | uint32_t(bp);
      if (left0 && !left1) {
        const double s = left_sign(t, m) * t.c;
        auto it = ent.find(pk);
        if (it == ent.end()) {
          ent.emplace(pk, Entry{{s * f[0], s * f[1], s * f[2], s * f[3]}, false});
        } else {
          for (int e = 0; e < 4; ++e) it->second.f[e] += s * f[e];
        }
      } else {
        if (!left0 && left1) { errors[m] = "right-keyed state turned left-keyed"; break; }
        M2 g = f;
        if (left0) {
          const double s = left_sign(t, m) * left_sign(t, m + 1);
          for (double& e : g) e *= s;
        }
        auto it = ent.find(pk);
        if (it == ent.end()) {
          ent.emplace(pk, Entry{g, true});
        } else if (it->second.f != g) {
          errors[m] = "inconsistent pass-through factor";
          break;
        }
      }
    }
    // deterministic order: by (b_out, s_out, b_in, s_in)
    std::vector<std::pair<uint64_t, M2>> list;
    list.reserve(ent.size());
    for (auto& kv : ent) list.emplace_back(kv.first, kv.second.f);
    std::sort(list.begin(), list.end(), [](const auto& a, const auto& b) {
      const uint32_t ao = uint32_t(a.first), bo = uint32_t(b.first);
      return ao != bo ? ao < bo : a.first < b.first;
    });
    MpoSite st;
    st.w_in = mpo.w[m];
    st.w_out = mpo.w[m + 1];
    for (auto& e : list) {
      const int b = int(e.first >> 32), bp = int(uint32_t(e.first));
      for (int so = 0; so < 2; ++so)
        for (int si = 0; si < 2; ++si) {
          const double val = e.second[so * 2 + si];
          if (val == 0.0) continue;
          if (mpo.charge[m + 1][bp] - mpo.charge[m][b] != so - si) {
            errors[m] = "transition violates particle-number charge";
            continue;
          }
          st.b_in.push_back(b);
          st.b_out.push_back(bp);
          st.s_out.push_back(uint8_t(so));
          st.s_in.push_back(uint8_t(si));
          st.val.push_back(val);
        }
    }
    mpo.site[m] = std::move(st);
  }
  for (int m = 0; m < L; ++m)
    if (!errors[m].empty()) throw std::runtime_error("build_mpo: site " + std::to_string(m) + ": " + errors[m]);
  return mpo;
}

}  // namespace pv

namespace pv {
void mpo_to_dense(const Mpo& mpo, double* out) {
  const int L = mpo.L;
  if (L > 8) throw std::runtime_error("mpo_to_dense: L > 8");
  // ops[b] is a dim x dim row-major matrix over the first m orbitals
  std::vector<std::vector<double>> ops(1, std::vector<double>(1, 1.0));
  for (int m = 0; m < L; ++m) {
    const int d = 1 << m, d2 = 2 * d;
    const MpoSite& st = mpo.site[m];
    std::vector<std::vector<double>> nxt(st.w_out, std::vector<double>(size_t(d2) * d2, 0.0));
    for (size_t e = 0; e < st.val.size(); ++e) {
      const auto& O = ops[st.b_in[e]];
      auto& R = nxt[st.b_out[e]];
      const int so = st.s_out[e], si = st.s_in[e];
      const double val = st.val[e];
      // new orbital m is the most significant bit: index = x + s * 2^m
      for (int x = 0; x < d; ++x)
        for (int y = 0; y < d; ++y)
          R[size_t(x + so * d) * d2 + (y + si * d)] += val * O[size_t(x) * d + y];
    }
    ops = std::move(nxt);
  }
  const size_t n = size_t(1) << L;
  for (size_t i = 0; i < n * n; ++i) out[i] = ops[0][i];
}
}  // namespace pv
