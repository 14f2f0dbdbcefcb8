// FP32 GEMM kernels (v_mfma_f32_32x32x2_f32).
#define FMD_GEMM_T float
#include "gemm_inst.h"
