// lbm_instances.hpp -- the kernel templates instantiated for one storage
// format.  LBM_INSTANCES(PREFIX, ST) expands to PREFIX-qualified explicit
// instantiations: `template` in the translation unit that compiles them
// (lbm_kern.hip, once per storage), `extern template` in the host
// translation unit, which launches them.  Kernel variants: every
// combination of the option bits except the reduced collision together with
// the explicit equilibrium.
#pragma once

#define LBM_INST_VARIANT(PREFIX, ST, V)                                                                        \
    PREFIX __global__ void k_stream_collide<ST, V, true>(KDomain, const TileRec *, uint32_t);                 \
    PREFIX __global__ void k_stream_collide<ST, V, false>(KDomain, const TileRec *, uint32_t);                \
    PREFIX __global__ void k_local_collide<ST, V>(KDomain, const TileRec *, uint32_t);                        \
    PREFIX __global__ void k_collide_batched<ST, V, 0u>(const KDomain *, const TileRec *, const TileRec *,     \
                                                        const uint32_t *, uint32_t);                            \
    PREFIX __global__ void k_collide_batched<ST, V, 1u>(const KDomain *, const TileRec *, const TileRec *,     \
                                                        const uint32_t *, uint32_t);

#define LBM_INSTANCES(PREFIX, ST)                                                                              \
    LBM_INST_VARIANT(PREFIX, ST, 0)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 1)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 2)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 3)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 4)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 5)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 6)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 7)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 8)                                                                            \
    LBM_INST_VARIANT(PREFIX, ST, 10)                                                                           \
    LBM_INST_VARIANT(PREFIX, ST, 12)                                                                           \
    LBM_INST_VARIANT(PREFIX, ST, 14)                                                                           \
    PREFIX __global__ void k_normalise<ST>(KDomain, const TileRec *, uint32_t);                               \
    PREFIX __global__ void k_side_refresh<ST>(KDomain);                                                       \
    PREFIX __global__ void k_curved_refresh<ST>(KDomain, const TileRec *, uint32_t);                          \
    PREFIX __global__ void k_init_eq<ST>(KDomain, const float *, const float *);                              \
    PREFIX __global__ void k_moments<ST>(KDomain, float *, float *);                                          \
    PREFIX __global__ void k_export<ST>(KDomain, float *);                                                    \
    PREFIX __global__ void k_import<ST>(KDomain, const float *);
