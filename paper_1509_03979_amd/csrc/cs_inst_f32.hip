// FP32 transform kernels for every four-step shape.
#define CS_T float
#define CS_T_IS_F64 0
#include "cs_inst.inc"
