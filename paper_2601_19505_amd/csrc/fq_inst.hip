// fq_inst.hip -- instantiations of the merge and spawn kernels for one
// (address words, model variant) pair, chosen by FQ_INST_W and
// FQ_INST_MODEL at compile time (the build compiles this file once per pair).
#include <hip/hip_runtime.h>

#include "fq_kernels.hpp"

#if !defined(FQ_INST_W) || !defined(FQ_INST_MODEL)
#error "compile with -DFQ_INST_W=<1|2> -DFQ_INST_MODEL=<0..3>"
#endif

FQ_STEP_KERNEL_SET(, FQ_INST_W, FQ_INST_MODEL)
