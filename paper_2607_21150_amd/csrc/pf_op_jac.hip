// One apply mode of the FP64 operator dispatch, compiled as its own unit.
#include "pf_dispatch.hpp"

template pf_status dispatch_op64<pfmf::M_JAC>(pf_ctx*, pfmf::OpArgs, hipStream_t);
