// Tree (TSQR) Householder QR of a tall-skinny matrix by 32-column panels
// (tsqr.hip): the factored form kept between the factorisation and the
// application of Q.  Every level shrinks the rows by 288 / 32 = 9, so eight
// levels cover any matrix that fits in memory.
#pragma once

#include "common.h"

namespace dme {

constexpr int kTsqrMaxLevels = 8;

struct TsqrLevel {
  int64_t M = 0;          // rows of this level's matrix
  int G = 0;              // blocks
  double* mat = nullptr;  // level 0: the panel in W; level >= 1: stacked R factors (M x pb, ld M)
  int64_t ld = 0;
  double* T = nullptr;    // G blocks of 32 x 32 compact-WY factors (column-major)
};

struct TsqrPanel {
  int64_t c0 = 0;
  int pb = 0;
  int nlev = 0;
  TsqrLevel lev[kTsqrMaxLevels];
};

// The factored panels of one QR; pointers into the caller's workspace.
struct TsqrState {
  int64_t n = 0, k = 0, ld = 0;
  double* W = nullptr;
  std::vector<TsqrPanel> panels;
};

// Whether the tree QR serves an n x k matrix (any n, k >= 1).
bool tsqr_supported(int64_t n, int64_t k);
// Workspace (bytes) of tsqr_factor for n x k.
size_t tsqr_workspace(int64_t n, int64_t k);
// W (n x k, ld n) = Q R: R in W's upper triangle (rows < min(n, k)); the
// reflectors stay in W and in `ws`, described by `st`.
void tsqr_factor(hipStream_t s, int64_t n, int64_t k, double* W, TsqrState& st, Arena& ws);
// X (n x ncols, ld ldx) <- Q X.
void tsqr_apply_q(hipStream_t s, const TsqrState& st, double* X, int64_t ldx, int64_t ncols);

}  // namespace dme
