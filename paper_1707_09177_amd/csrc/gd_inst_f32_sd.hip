// Solve kernels for float fields, solver GD_STEEPEST_DESCENT.
#define GD_T float
#define GD_SOLVER GD_STEEPEST_DESCENT
#define GD_FN solve_kernels_f32_sd
#include "gd_inst.inc"
