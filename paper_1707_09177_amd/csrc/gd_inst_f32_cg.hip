// Solve kernels for float fields, solver GD_CG.
#define GD_T float
#define GD_SOLVER GD_CG
#define GD_FN solve_kernels_f32_cg
#include "gd_inst.inc"
