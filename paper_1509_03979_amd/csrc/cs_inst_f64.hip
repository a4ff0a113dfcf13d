// FP64 transform kernels for every four-step shape.
#define CS_T double
#include "cs_inst.inc"
