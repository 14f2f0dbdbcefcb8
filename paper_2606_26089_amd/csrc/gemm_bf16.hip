// BF16-operand GEMM kernels with FP32 accumulation (v_mfma_f32_32x32x16_bf16).
#define FMD_GEMM_T bf16
#include "gemm_inst.h"
