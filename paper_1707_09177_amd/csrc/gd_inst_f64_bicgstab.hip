// Solve kernels for double fields, solver GD_BICGSTAB.
#define GD_T double
#define GD_SOLVER GD_BICGSTAB
#define GD_FN solve_kernels_f64_bicgstab
#include "gd_inst.inc"
