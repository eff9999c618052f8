// Solve kernels for double fields, solver GD_CG.
#define GD_T double
#define GD_SOLVER GD_CG
#define GD_FN solve_kernels_f64_cg
#include "gd_inst.inc"
