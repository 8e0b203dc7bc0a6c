/*
 * gp_cpu.h -- C ABI of the host (CPU) implementation of the two refinements.
 *
 * The multi-core and SIMD CPU designs of Zhang & You (arXiv 1403.0802, Sec. III.B-C,
 * compared in Tables 2-5): points of a grid cell are refined against the cell's
 * candidate features, one core per cell (multi-core) and eight points per AVX-512
 * instruction (SIMD: the points-to-lanes mapping the paper uses on its vector units).
 * It exists for the host-side comparison next to the GPU library (libgp.so); it is
 * not on the GPU path.
 *
 * Definitions, grid and results are those of gp.h: FP64 with the operation order
 * stated there and no fused multiply-add, so every mode returns the same bits as the
 * GP_FP64 form of the GPU library.
 */
#ifndef GP_CPU_H
#define GP_CPU_H

#include <stdint.h>

#include "gp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Execution modes, the axes of the paper's CPU tables. */
#define GP_CPU_SC 0       /* one core, scalar */
#define GP_CPU_MC 1       /* all cores (OpenMP over cells), scalar */
#define GP_CPU_SC_SIMD 2  /* one core, AVX-512 (8 FP64 points per instruction) */
#define GP_CPU_MC_SIMD 3  /* all cores, AVX-512 */

typedef struct gp_cpu_stats {
    uint64_t tests;      /* point-edge tests: sum over cells npts * sum nedges(cands) */
    int32_t threads;     /* threads used by the refinement */
    int32_t simd;        /* 1 if the AVX-512 code ran (0: the host lacks AVX-512F/DQ
                            and a SIMD mode ran scalar) */
    double ms_filter;    /* grid build and point pairing */
    double ms_refine;    /* refinement */
} gp_cpu_stats;

/* Full join on HOST arrays: builds the grid of *params for the features (as
 * gp_build_grid does: MBBs expanded by D for P2P, padded by cs*2^-20, rasterised,
 * candidate lists by ascending id), pairs the n points by cell and refines them.
 * kind GP_PIP writes out_id; GP_P2P writes out_id and out_dist.  threads <= 0 uses
 * every OpenMP thread in the MC modes.  Synchronous.  GP_E_INVALID_ARG for bad
 * arguments, GP_E_BAD_GEOMETRY for malformed offsets or short polylines,
 * GP_E_CAPACITY for grids above 2^28 cells. */
gp_status gp_cpu_join(gp_kind kind, const gp_geometry *geom, const gp_grid_params *params,
                      int64_t n, const double *px, const double *py, int32_t *out_id,
                      double *out_dist, int32_t mode, int32_t threads, gp_cpu_stats *stats);

/* 1 if this host can run the AVX-512 modes. */
int32_t gp_cpu_has_simd(void);

#ifdef __cplusplus
}
#endif

#endif /* GP_CPU_H */
