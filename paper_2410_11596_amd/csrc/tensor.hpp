// Construction kernels (double layer, basis change, initial environment, dots).
#pragma once
#include <cmath>
#include <vector>

#include "hctm_internal.hpp"

namespace hctm {

// Rows of the leg basis as a table: row a of U has the plain indices
// ti[2a], ti[2a+1] (-1 if absent) with coefficients tc[2a], tc[2a+1].
// rotated: the eigenbasis of the bra-ket swap (Sec. II B; even sector first:
// |k k>, then (|k l> + |l k>)/sqrt2 for k < l; odd: (|k l> - |l k>)/sqrt2);
// otherwise the identity.  tti/ttc: the same table for U^T.
inline void basis_table(int D, bool rotated, std::vector<int>& ti, std::vector<double>& tc, std::vector<int>& tti,
                        std::vector<double>& ttc) {
  const int q = D * D;
  ti.assign(2 * q, -1);
  tti.assign(2 * q, -1);
  tc.assign(2 * q, 0.0);
  ttc.assign(2 * q, 0.0);
  if (rotated) {
    const double r2 = 1.0 / std::sqrt(2.0);
    int row = 0;
    for (int k = 0; k < D; ++k) {
      ti[2 * row] = k * D + k;
      tc[2 * row] = 1.0;
      ++row;
    }
    for (int sgn = 0; sgn < 2; ++sgn)
      for (int k = 0; k < D; ++k)
        for (int l = k + 1; l < D; ++l) {
          ti[2 * row] = k * D + l;
          tc[2 * row] = r2;
          ti[2 * row + 1] = l * D + k;
          tc[2 * row + 1] = sgn ? -r2 : r2;
          ++row;
        }
  } else {
    for (int a = 0; a < q; ++a) {
      ti[2 * a] = a;
      tc[2 * a] = 1.0;
    }
  }
  std::vector<int> cnt(q, 0);
  for (int a = 0; a < q; ++a)
    for (int w = 0; w < 2; ++w) {
      const int K = ti[2 * a + w];
      if (K < 0) continue;
      tti[2 * K + cnt[K]] = a;
      ttc[2 * K + cnt[K]] = tc[2 * a + w];
      ++cnt[K];
    }
}

constexpr int kMaxPairs = 16;
struct DLArgs {
  const double* A;        // d x D^4 single-layer tensors, [s,u,l,d,r]
  double* out;            // q^4 plain, rotated basis
  const int* tab_idx;     // basis table: row a -> (K0, K1), -1 if absent
  const double* tab_c;    // coefficients
  int d, D;
  int npairs;
  int ket[kMaxPairs], bra[kMaxPairs];
  double w[kMaxPairs];
};
void double_layer_basis(const DLArgs& g, hipStream_t s);
void basis4(const double* in, double* out, int q, const int* tab_idx, const double* tab_c, hipStream_t s);
void init_env(const double* a, int q, int rot, const double* b, const int* tab_idx, const double* tab_c, double* C,
              double* T, hipStream_t s);

struct DotJob {
  const double* x;
  const double* y;
  long long n;
  double* out;
};
constexpr int kMaxDots = 32;
struct DotBatch {
  DotJob j[kMaxDots];
  int n;
};
// scratch: 64 doubles per job of a batch (64 * kMaxDots)
void dots(const std::vector<DotJob>& jobs, double* scratch, hipStream_t s);

// rho (n x n) from precomputed dot products, divided by its trace.
// mode 0: rho1, dots[s*d + s'] (dense) ; mode 1: rho1 Z2, dots over s <= s'
// mode 2: rho2 dense, dots[(s1 d + s1') d^2 + (s2 d + s2')]
// mode 3: rho2 Z2, dots of sym-sym and anti-anti pairs (see tensor.hip)
void assemble_rho(const double* dots, int d, int mode, double* rho, hipStream_t s);
// Complex (Hermitian) RDM from real dot products of structured tensors.
// One site (two_site = 0): per pair s <= s' (pair_le order) four dots
//   [eps_re . S1_re, eps_im . S1_im, eps_re . S2_re, eps_im . S2_im] of the
// structured parts of the impurity S1 + i S2, rho[s][s'] = <eps, S1> +
// i <eps, S2> = (t0 - t1) + i (t2 - t3).
// Two sites: per (s1 s1', s2 s2') eight dots of the halves L1, L2 (left) and
// R1, R2 (right), [L1.R1 re, L1.R1 im, L2.R2 re, L2.R2 im, L1.R2 re,
// L1.R2 im, L2.R1 re, L2.R1 im] (re, im: the dot of the parts), with
// <X, Y> = re - im; rho = <L1,R1> - <L2,R2> + i (<L1,R2> + <L2,R1>).
// The lower triangle is the conjugate of the upper, the result is divided
// by its trace; re and im are n x n (n = d or d^2), device memory.
void assemble_rho_complex(const double* dots, int d, int two_site, double* re, double* im, hipStream_t s);
// e = sum_k Tr(rho_k h), k over nrho matrices of size n x n
void trace_products(const double* rho, int nrho, const double* h, int n, double* e, hipStream_t s);
// num = ||x - S x||^2, den = ||x + S x||^2 with S the bra-ket swap on every
// leg of a plain q^4 tensor (q = D^2); out = sqrt(num / den)
void swap_asym(const double* x, int D, double* part, double* out, hipStream_t s);
// out = sum of the diagonals of a list of square blocks
void trace_blocks(const double* const* p, const int* n, const int* ld, int nb, double* out, hipStream_t s);
// out = ln|z[0]| + ln|z[1]| - ln|z[2]| - ln|z[3]|
void log_ratio(const double* z, double* out, hipStream_t s);

}  // namespace hctm
