// FP64 transform kernels for every four-step shape.
#define CS_T double
#define CS_T_IS_F64 1
#include "cs_inst.inc"
