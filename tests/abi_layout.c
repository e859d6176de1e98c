/* Prints the byte layout of the public structs of include/fde.h, compiled with the system C
 * compiler; the CPU tests compare it with the ctypes declarations of the Python binding. */
#include <stddef.h>
#include <stdio.h>

#include "fde.h"

#define F(T, m) printf("%s.%s %zu\n", #T, #m, offsetof(T, m))
int main(void) {
  printf("fde_problem %zu\n", sizeof(fde_problem));
  F(fde_problem, alpha); F(fde_problem, beta); F(fde_problem, n1); F(fde_problem, n2);
  F(fde_problem, a1); F(fde_problem, b1); F(fde_problem, a2); F(fde_problem, b2);
  F(fde_problem, tau); F(fde_problem, precision); F(fde_problem, mg_variant);
  F(fde_problem, omega); F(fde_problem, nu_pre); F(fde_problem, nu_post);
  F(fde_problem, coarsest_n); F(fde_problem, restart); F(fde_problem, maxit); F(fde_problem, rtol);
  printf("fde_stats %zu\n", sizeof(fde_stats));
  F(fde_stats, iters); F(fde_stats, restarts); F(fde_stats, converged);
  F(fde_stats, relres_true); F(fde_stats, relres_est);
  return 0;
}
