// LOBPCG driver (placeholder until the block kernels land).
#include "kc_state.h"

namespace kc {

struct SolverWork {
  int dummy = 0;
};

void solver_release(kc_op* op) {
  delete op->solver;
  op->solver = nullptr;
}

}  // namespace kc

extern "C" {

void kc_solve_opts_default(kc_solve_opts* o) {
  if (!o) return;
  o->m = 10;
  o->guard = 0;
  o->tol = 1e-8;
  o->maxit = 500;
  o->prec = KC_PREC_FP64;
  o->switch_tol = 1e-3;
  o->batch_k = 1;
  o->seed = 1234;
  o->verbose = 0;
}

int kc_solve(kc_op* op, int ik0, int nk, const kc_solve_opts* opts, double* eig_host, double* res_host,
             int* iters_host, void* X_out, void* stream) {
  KC_ARG(op != nullptr && opts != nullptr, "NULL op or opts");
  (void)ik0; (void)nk; (void)eig_host; (void)res_host; (void)iters_host;
  (void)X_out; (void)stream;
  kc::set_error("kc_solve not built yet");
  return KC_ERR_UNSUPPORTED;
}

}  // extern "C"
