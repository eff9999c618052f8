// Solve kernels for float fields, solver GD_VANCITTERT.
#define GD_T float
#define GD_SOLVER GD_VANCITTERT
#define GD_FN solve_kernels_f32_vc
#include "gd_inst.inc"
