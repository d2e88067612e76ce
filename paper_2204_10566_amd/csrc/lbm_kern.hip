// lbm_kern.hip -- compiles the kernels of one storage format
// (LBM_KERN_ST = 0 FP32, 1 FP16S, 2 BF16S) into their own object, so that
// the three formats build in parallel; lbm.hip launches them.
#include "lbm_device.hpp"
#include "lbm_instances.hpp"

#ifndef LBM_KERN_ST
#error "LBM_KERN_ST must name the storage format"
#endif

namespace lbm {
LBM_INSTANCES(template, LBM_KERN_ST)
} // namespace lbm
