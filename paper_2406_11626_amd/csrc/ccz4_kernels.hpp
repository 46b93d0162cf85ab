// Launchers of the device kernels (implemented in ccz4_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ccz4_algebra.hpp"
#include "ccz4_layout.hpp"

namespace ccz4 {

struct InitArgs {
    double sp[16];
};

hipError_t launch_init(double *Q, const PatchGeom *geom, const uint8_t *bmask, int32_t npatch, int32_t scen,
                       const InitArgs &a, hipStream_t st);
hipError_t launch_fill(double *Q, const FaceTask *tasks, int32_t ntask, int32_t transfer, hipStream_t st);
// right-hand side / fused stage launch configurations: bit 0 selects the LDS-staged kernel (else
// the phased one), bit 1 the plain block order (else the XCD-grouped order), bits 2-3 the order in
// which the launch walks the leaves (the permutations of the context, KV_ORDERS of them)
enum KernelVariant : int32_t { KV_PHASED = 0, KV_LDS = 1, KV_LINEAR = 2, KV_ORDER_SHIFT = 2, KV_ORDERS = 4,
                               KV_COUNT = 16 };

// order: the leaf that the launch's logical patch index q takes is order[q] (a permutation)
hipError_t launch_rhs(const double *Q, double *K, const PatchGeom *geom, int32_t npatch, const RhsParams &p,
                      int32_t precision, int32_t variant, const int32_t *order, const BoundaryFace *bf,
                      const double *bg, int32_t nbf, const int32_t *pface, hipStream_t st);
hipError_t launch_stage(int32_t s, double dt, const double *Qs, const double *Qn, double *acc, double *Qx,
                        const PatchGeom *geom, int32_t npatch, const RhsParams &p, int32_t precision,
                        int32_t variant, const int32_t *order, const BoundaryFace *bf, const double *bg, int32_t nbf,
                        const int32_t *pface, const int32_t *nbr, int32_t paxes, const int32_t *gnbr,
                        hipStream_t st);
hipError_t launch_rhs_sommerfeld(const double *Q, double *K, const PatchGeom *geom, const BoundaryFace *bf,
                                 const double *bg, int32_t nbf, int32_t frozen, hipStream_t st);
hipError_t launch_capture_bg(const double *Q, const BoundaryFace *bf, double *bg, int32_t nbf, hipStream_t st);
hipError_t launch_rk4(int32_t s, double dt, const double *Qn, const double *K, double *acc, double *Qx,
                      int32_t npatch, const BoundaryFace *bf, int32_t nbf, hipStream_t st);
hipError_t launch_regrid(const double *Qo, double *Qn, const RegridTask *tasks, int32_t n, hipStream_t st);
hipError_t launch_reconstruct(double *Q, const PatchGeom *geom, int32_t npatch, const int32_t *nbr, int32_t paxes,
                              const int32_t *gnbr, hipStream_t st);
hipError_t launch_tracers(const double *Q, const PatchGeom *geom, int32_t npatch, int64_t n, double *pos,
                          const TracerSlots &sl, const LeafLookup &lk, double *out, double dt, int32_t advance, hipStream_t st);
hipError_t launch_tag_tracers(const TrackBox *box, int32_t npatch, int64_t n, const double *pos, const TrackRadii &R,
                              int32_t max_level, int8_t *tags, hipStream_t st);
int64_t constraints_blocks(int32_t npatch);
hipError_t launch_constraints(const double *Q, double *HM, const PatchGeom *geom, int32_t npatch,
                              double r_excise, double *part, double *out3, hipStream_t st);
hipError_t launch_tags(const double *Q, const double *HM, const PatchGeom *geom, const int32_t *sib,
                       int32_t npatch, double theta_r, double theta_c, int32_t max_level, int8_t *tags,
                       double *ind, hipStream_t st);

}  // namespace ccz4
