/* Plain-C use of the library's ABI (no Python, no GPU needed for these calls): describe a
 * one-wedge mesh, let fo_mesh_create reject an invalid variant of it, and print the status
 * strings.  Build: gcc -Iinclude abi_check.c -Lpaper_2204_04321_amd -lfo_stokes */
#include <stdio.h>
#include <string.h>

#include "fo_stokes.h"

int main(void) {
  double xy[6] = {0.0, 0.0, 1000.0, 0.0, 0.0, 800.0};
  int32_t cells[3] = {0, 1, 2};
  double s[3] = {900.0, 900.0, 900.0}, H[3] = {500.0, 500.0, 500.0}, beta[3] = {100.0, 100.0, 100.0};
  fo_mesh_desc d;
  memset(&d, 0, sizeof d);
  d.elem = FO_WEDGE6;
  d.n_base_verts = 3;
  d.n_base_cells = 1;
  d.n_layers = 2;
  d.base_xy = xy;
  d.base_cells = cells;
  d.surface = s;
  d.thickness = H;
  d.beta = beta;
  d.sigma = NULL;
  d.A = 1e-16; d.n = 3.0; d.rho = 910.0; d.g = 9.81; d.eps0 = 1e-10;

  fo_mesh *m = NULL;
  H[1] = -1.0;   /* invalid thickness: rejected on the host */
  fo_status st = fo_mesh_create(&d, NULL, &m);
  printf("create with H < 0: %d (%s): %s\n", (int)st, fo_status_string(st), fo_last_error());
  if (st != FO_EDEGENERATE || m != NULL) return 1;

  H[1] = 500.0;
  cells[1] = 2; cells[2] = 1;   /* clockwise */
  st = fo_mesh_create(&d, NULL, &m);
  printf("create with a clockwise cell: %d (%s)\n", (int)st, fo_status_string(st));
  if (st != FO_EDEGENERATE) return 1;

  st = fo_assemble_residual(NULL, NULL, NULL, NULL);
  printf("residual on a NULL mesh: %d (%s)\n", (int)st, fo_status_string(st));
  if (st != FO_EINVAL) return 1;
  fo_newton_opts o;
  fo_newton_default_opts(&o);
  printf("default Newton tol %g, restart %d, linear solver %d, opts size %d\n", o.tol, (int)o.gmres_restart,
         (int)o.linear_solver, (int)sizeof o);
  printf("learned init: fallback %d, smooth %d, report size %d\n", (int)o.learned_fallback, (int)o.learned_smooth,
         (int)sizeof(fo_newton_report));
  return 0;
}
