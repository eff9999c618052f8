// Solve kernels for double fields, solver GD_STEEPEST_DESCENT.
#define GD_T double
#define GD_SOLVER GD_STEEPEST_DESCENT
#define GD_FN solve_kernels_f64_sd
#include "gd_inst.inc"
