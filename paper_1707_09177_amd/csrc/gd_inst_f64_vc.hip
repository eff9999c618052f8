// Solve kernels for double fields, solver GD_VANCITTERT.
#define GD_T double
#define GD_SOLVER GD_VANCITTERT
#define GD_FN solve_kernels_f64_vc
#include "gd_inst.inc"
