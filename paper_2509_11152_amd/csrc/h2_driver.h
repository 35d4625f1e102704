// Host drivers behind the C ABI.
#pragma once
#include <vector>

#include "h2_internal.h"

namespace h2drv {

void matvec(h2_context_s* ctx, h2_matrix_s* H, const double* X, int64_t ldx, int nrhs, double* Y,
            int64_t ldy);

// the product with its work arrays in caller-provided device memory
void matvec_in(h2_context_s* ctx, h2_matrix_s* H, const double* X, int64_t ldx, int nrhs,
               double* Y, int64_t ldy, char* scratch, int64_t cap);

std::vector<h2_factor_s*> factor(h2_context_s* ctx, const std::vector<h2_matrix_s*>& Hs,
                                 double tol, h2_prec prec, const h2_factor_opts& opts);

void solve(h2_context_s* ctx, const std::vector<h2_factor_s*>& Fs,
           const std::vector<const double*>& B, const std::vector<int64_t>& ldb, int nrhs,
           const std::vector<double*>& X, const std::vector<int64_t>& ldx);

bool solve_ir(h2_context_s* ctx, h2_matrix_s* H, h2_factor_s* F, const double* B, int64_t ldb,
              int nrhs, double* X, int64_t ldx, const h2_ir_opts& o, h2_ir_report& rep);

}  // namespace h2drv
