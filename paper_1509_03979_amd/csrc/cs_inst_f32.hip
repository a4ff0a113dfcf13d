// FP32 transform kernels for every four-step shape.
#define CS_T float
#include "cs_inst.inc"
