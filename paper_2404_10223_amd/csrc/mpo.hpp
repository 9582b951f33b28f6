// Matrix-product operator of the electronic Hamiltonian, built on the host.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

namespace tnqe {

// Nonzeros of a local 4x4 operator (bra index kp, ket index k), entries +-1.
struct OpPattern {
  int n = 0;
  int kp[4] = {0, 0, 0, 0};
  int k[4] = {0, 0, 0, 0};
  double f[4] = {0, 0, 0, 0};
};

// Transitions of one site between a channel class at the left bond and one at
// the right bond that share one local operator, as a CSR matrix
// [channels of cout] x [channels of cin].  A nonzero's value is either fixed
// (1) or a coefficient slot filled per basis.
struct MpoGroup {
  int cin = 0, cout = 0, pattern = 0;
  std::vector<int> rowptr, col, slot;   // sparse form; slot < 0: fixed value 1
  // dense form (coefficient couplings between whole channel ranges): a block
  // of rows [r0, r0 + nr) x columns [c0, c0 + nc), row-major, slot per entry
  // (-1: zero, -2: fixed value 1); when dense, rowptr/col/slot are empty
  bool dense = false;
  int r0 = 0, nr = 0, c0 = 0, nc = 0;
  std::vector<int> dslot;
  int64_t val_off = 0;                  // offset of the group's values in its site
  int64_t nvals() const { return dense ? (int64_t)nr * nc : (int64_t)slot.size(); }
};

struct MpoClass {
  int da = 0, db = 0;   // shift bra sector - ket sector
  int nw = 0;           // channels
};

struct MpoStructure {
  int N = 0;
  std::vector<std::vector<MpoClass>> classes;   // per bond
  std::vector<std::vector<MpoGroup>> groups;    // per site
  std::vector<OpPattern> patterns;
  int64_t nslot = 0;                            // coefficient slots
  std::vector<int> term_slot;                   // per term, in enumeration order
  std::vector<double> term_factor;              // sort sign x 1 or 1/2
  int final_class = 0, final_H = 0, final_I = 0;
  std::vector<int> I_class, I_loc;              // per bond: class and index of the channel I
  int max_bond = 0;
  std::vector<int64_t> site_nnz, site_nnz_off;  // CSR sizes per site and offsets
};

// Channel structure for N sites; independent of the integral values.
void mpo_build_structure(int N, MpoStructure &m);

// CSR values of all sites, concatenated in site order (group order inside a
// site), for one-electron integrals h [N][N] and (pq|rs) g [N^4].
void mpo_values(const MpoStructure &m, const double *h, const double *g, std::vector<double> &vals,
                std::vector<double> &slotval_scratch);

}  // namespace tnqe
