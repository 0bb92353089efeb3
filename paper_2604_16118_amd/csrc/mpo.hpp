// Symbolic matrix product operator of H = T + V built on the host.
//
// H = sum_ij h_ij a_i^* a_j + sum_{i<j,k<l} w_ijkl a_i^* a_j^* a_k a_l with
// w_ijkl = v_ijkl - v_jikl - v_ijlk + v_jilk, the antisymmetrised form of the two-body
// sum of Section 1.1 (eq. hamil), which is equal to it by the anticommutation relations.
//
// Every term is a product of Jordan-Wigner operators a_i = S x..x S x A x I x..x I, so its
// restriction to the sites left of a cut and the factor on each single site are exact
// Kronecker factors.  At each cut a term is keyed either by its operators left of the
// cut ("left-normal" bond state) or by those right of it ("complementary" state); the
// choice follows the counting behind the rank bounds of Thm. opranks (the side with
// fewer operators, ties to the left in the left half of the chain).  Bond states are
// grouped by their particle-number change q in {-2..2}, so the operator is block-sparse
// in the same sense as the MPS blocks of Section 2.3.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

namespace pv {

struct MpoSite {
  int w_in = 0, w_out = 0;
  // transitions b_in -> b_out with local operator entry <s_out| f |s_in> = val
  std::vector<int32_t> b_in, b_out;
  std::vector<uint8_t> s_out, s_in;
  std::vector<double> val;
};

struct Mpo {
  int L = 0;
  std::vector<int> w;                        // bond dimension at cut m = 0..L
  std::vector<std::vector<int8_t>> charge;   // charge[m][b]
  std::vector<std::array<int, 6>> qoff;      // qoff[m][q+2] .. qoff[m][q+3]: states of charge q
  std::vector<MpoSite> site;                 // site[k] acts on orbital k (0-based), cuts k -> k+1
  int64_t n_terms = 0;
};

// Build the operator for L orbitals; h is L*L row-major, v is L^4 row-major
// (v[((i*L+j)*L+k)*L+l] multiplies a_i^* a_j^* a_k a_l).  Throws std::runtime_error on
// inconsistent input.  diag_shift is added to every h_ii (gamma/N turns H into H + gamma
// on the N-particle space, as in Section 7.1.1).
Mpo build_mpo(int L, const double* h, const double* v, double diag_shift);

}  // namespace pv

namespace pv {
// Dense 2^L x 2^L matrix (row-major; index bit i = occupation of orbital i+1) of the
// operator, by the left recursion O_{b'}(m+1) = sum_b O_b(m) (x) W_m[b,b'].  For tests,
// L <= 8.
void mpo_to_dense(const Mpo& mpo, double* out);
}  // namespace pv
