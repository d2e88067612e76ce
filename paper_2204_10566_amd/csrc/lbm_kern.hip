// lbm_kern.hip -- compiles the kernels of one storage format
// (LBM_KERN_ST = 0 FP32, 1 FP16S, 2 BF16S) into their own object, so that
// the formats build in parallel; lbm.hip launches them.  LBM_KERN_WIDE = 1
// compiles the step kernels of arrays past 4 GiB instead.
#include "lbm_device.hpp"
#include "lbm_instances.hpp"

#ifndef LBM_KERN_ST
#error "LBM_KERN_ST must name the storage format"
#endif

namespace lbm {
#if LBM_KERN_WIDE
LBM_INSTANCES_WIDE(template, LBM_KERN_ST)
#else
LBM_INSTANCES(template, LBM_KERN_ST)
#endif
} // namespace lbm
