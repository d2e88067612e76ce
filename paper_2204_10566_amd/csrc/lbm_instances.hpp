// lbm_instances.hpp -- the kernel templates instantiated for one storage
// format.  LBM_INSTANCES(PREFIX, ST) and LBM_INSTANCES_WIDE(PREFIX, ST)
// expand to PREFIX-qualified explicit instantiations: `template` in the
// translation unit that compiles them (lbm_kern.hip, once per storage and
// addressing width), `extern template` in the host translation unit, which
// launches them.  Kernel variants: every combination of the option bits
// except the reduced collision together with the explicit equilibrium.
// The wide set holds the single-domain step kernels of arrays past 4 GiB.
#pragma once

#define LBM_FOR_VARIANTS(M, PREFIX, ST)                                                                        \
    M(PREFIX, ST, 0)                                                                                           \
    M(PREFIX, ST, 1)                                                                                           \
    M(PREFIX, ST, 2)                                                                                           \
    M(PREFIX, ST, 3)                                                                                           \
    M(PREFIX, ST, 4)                                                                                           \
    M(PREFIX, ST, 5)                                                                                           \
    M(PREFIX, ST, 6)                                                                                           \
    M(PREFIX, ST, 7)                                                                                           \
    M(PREFIX, ST, 8)                                                                                           \
    M(PREFIX, ST, 10)                                                                                          \
    M(PREFIX, ST, 12)                                                                                          \
    M(PREFIX, ST, 14)

#define LBM_INST_VARIANT(PREFIX, ST, V)                                                                        \
    PREFIX __global__ void k_stream_collide<ST, V, true, false>(KDomain, const TileRec *, uint32_t);          \
    PREFIX __global__ void k_stream_collide<ST, V, false, false>(KDomain, const TileRec *, uint32_t);         \
    PREFIX __global__ void k_local_collide<ST, V, false>(KDomain, const TileRec *, uint32_t);                 \
    PREFIX __global__ void k_collide_batched<ST, V, 0u, false>(const KDomain *, const TileRec *, uint32_t,      \
                                                               const uint32_t *, uint32_t);                     \
    PREFIX __global__ void k_collide_batched<ST, V, 0u, true>(const KDomain *, const TileRec *, uint32_t,       \
                                                              const uint32_t *, uint32_t);                      \
    PREFIX __global__ void k_collide_batched<ST, V, 1u, false>(const KDomain *, const TileRec *, uint32_t,      \
                                                               const uint32_t *, uint32_t);

#define LBM_INST_WIDE_VARIANT(PREFIX, ST, V)                                                                   \
    PREFIX __global__ void k_stream_collide<ST, V, true, true>(KDomain, const TileRec *, uint32_t);           \
    PREFIX __global__ void k_stream_collide<ST, V, false, true>(KDomain, const TileRec *, uint32_t);          \
    PREFIX __global__ void k_local_collide<ST, V, true>(KDomain, const TileRec *, uint32_t);

#define LBM_INSTANCES(PREFIX, ST)                                                                              \
    LBM_FOR_VARIANTS(LBM_INST_VARIANT, PREFIX, ST)                                                             \
    PREFIX __global__ void k_normalise<ST>(KDomain, const TileRec *, uint32_t);                               \
    PREFIX __global__ void k_side_refresh<ST>(KDomain);                                                       \
    PREFIX __global__ void k_curved_refresh<ST>(KDomain, const TileRec *, uint32_t);                          \
    PREFIX __global__ void k_init_eq<ST>(KDomain, const float *, const float *);                              \
    PREFIX __global__ void k_moments<ST>(KDomain, float *, float *);                                          \
    PREFIX __global__ void k_export<ST>(KDomain, float *);                                                    \
    PREFIX __global__ void k_import<ST>(KDomain, const float *);

#define LBM_INSTANCES_WIDE(PREFIX, ST) LBM_FOR_VARIANTS(LBM_INST_WIDE_VARIANT, PREFIX, ST)
