// Solve kernels for float fields, solver GD_BICGSTAB.
#define GD_T float
#define GD_SOLVER GD_BICGSTAB
#define GD_FN solve_kernels_f32_bicgstab
#include "gd_inst.inc"
