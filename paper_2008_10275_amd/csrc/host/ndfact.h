// Host-side factorisation of the mean-parameter preconditioner P (paper
// Sec. 4.2: P_T = A at the centre parameters; Sec. 5: the paper factorises it
// with a permuted LU).  Plain C++ (no HIP), so it can be tested on the CPU.
//
// P is reordered by nested dissection (recursive BFS-level bisection of the
// graph of P + P^T), which gives an elimination tree of supernodes: leaves are
// small subdomains, inner nodes are separators.  A multifrontal LU without
// pivoting factorises each front  [own | boundary]  densely.  The result is
// stored for a level-scheduled GPU solve in which every supernode's diagonal
// blocks are kept inverted:
//
//   forward  (L y = b, leaves first):  [y_own ; c] = Fw_s * f_own + [0 ; f_bnd]
//            Fw_s = [ L11^-1 ; -L21 L11^-1 ]          ((ns+nb) x ns)
//            f = b(own) + children's contribution rows c, assembled by index
//   backward (U x = y, root first):    x_own = Bw_s * [y_own ; x(bnd)]
//            Bw_s = [ U11^-1 | -U11^-1 U12 ]          (ns x (ns+nb))
//
// so that each level is one batch of dense products with no sequential chain
// inside a supernode.  P must have a nonsingular leading principal minor for
// every pivot (true when P + P^T is positive definite, as for the mean
// operator built from a convection-diffusion K_0 and PSD K_1, K_2).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace lrc {

struct CsrHost {
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct SupernodalFactor {
  int64_t n = 0;
  std::vector<int32_t> perm;    // new index -> original index
  std::vector<int32_t> iperm;   // original index -> new index
  int nsn = 0;                  // number of supernodes
  std::vector<int32_t> j0, ns, nb, parent, height, depth;
  std::vector<int64_t> bnd_off;          // nsn + 1
  std::vector<int32_t> bnd;              // boundary (new indices, ascending)
  // Dense blocks, column-major per supernode.
  std::vector<int64_t> fw_off, bw_off;   // nsn + 1
  std::vector<double> fw, bw;
  // Assembly of the forward front: front row p of supernode s has global id
  // front_off[s] + p (p < ns + nb); its sources are rows of the contribution
  // arena (supernode c owns rows cb_off[c] .. cb_off[c] + nb[c]).
  std::vector<int64_t> front_off, cb_off;   // nsn + 1
  std::vector<int64_t> asm_ptr;             // total_front_rows + 1
  std::vector<int64_t> asm_src;
  int nlev_fwd = 0, nlev_bwd = 0;
  // statistics
  int64_t max_front = 0;
  double dense_entries = 0.0;   // entries of all Fw + Bw blocks
  double factor_flops = 0.0;
  double seconds_order = 0.0, seconds_factor = 0.0, seconds_post = 0.0;
};

// Nested-dissection ordering only (exposed for tests): perm (new -> old) and the
// supernode tree (j0, ns, parent).  Returns false with *err on failure.
bool nd_order(const CsrHost& P, int leaf_size, std::vector<int32_t>* perm,
              std::vector<int32_t>* j0, std::vector<int32_t>* ns,
              std::vector<int32_t>* parent, std::string* err);

// Full factorisation.  Return codes: 0 ok, -1 invalid input, -4 zero/NaN pivot.
int nd_factor(const CsrHost& P, int leaf_size, int nthreads, SupernodalFactor* out,
              std::string* err);

}  // namespace lrc
