// The iteration kernels with FP32 accumulation in every reduction: the
// pure-FP32 precision ablation (sip_opts.reduce = SIP_F32).  Same source as
// the default FP64-accumulation build, in namespace sip::r32.
#define SIP_ACC float
#define SIP_KNS r32
#include "sip_kernels.hip"
