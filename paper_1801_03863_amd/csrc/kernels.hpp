// kernels.hpp -- launch interface between the host runtime and the HIP
// kernels of the fused stream-and-collide step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum Storage { ST_F64 = 0, ST_F32N64 = 1, ST_F32 = 2, ST_F16DEV = 3 };
enum Coll { CO_MINXENT4 = 0, CO_MINXENT2 = 1, CO_SRT = 2, CO_TRT = 3, CO_MRT = 4 };
enum Bc { BC_PERIODIC = 0, BC_TUBE = 1, BC_CAVITY = 2, BC_BOX = 3 };

// Status record of one instance (device memory).
struct DevStatus {
    uint32_t flags;
    int32_t pad;
    uint64_t first;  // (step << 32) | node of the first unstable node; all ones until then
    int64_t guarded;
};

// One lattice instance as the kernels see it.  Populations of instance i
// live in b planes of `plane` elements starting at element `offset` of each
// of the two buffers; node (x, y) is element y*pitch + x of a plane (D2Q9
// rows start on whole 128-byte lines; elements x >= nx of a row are padding
// that no kernel reads).  Node numbers (status, host fields) stay y*nx + x.
struct Inst {
    int32_t nx, ny;
    int32_t pitch;   // row stride in elements (>= nx)
    int64_t offset;
    int64_t plane;
    double omega;    // 1/tau
    double omega2;   // 1/tau2
    double u_lid;
    double rho0;
    double lid[9];   // equilibrium of (rho0, (u_lid, 0))
    int64_t stop;    // batched: the instance takes no step from this step index on
};

// Everything a step launch needs besides the buffers.
struct StepArgs {
    const Inst *inst;       // device table (batched) -- or nullptr
    Inst one;               // the single instance (non-batched launches)
    DevStatus *status;      // one record per instance
    const int64_t *step_base;  // if not null, added to `step` on the error path
    const int32_t *tile_inst;  // batched: instance of each tile
    const int32_t *tile_first; // batched: first node of each tile, or for two-step shapes the tile's index
                               // ty * tiles_x + tx within its instance
    int64_t step;
    int32_t bc;
    int32_t ntiles;
    int32_t tiles_x;        // single D2Q9: tiles along x
    int32_t xcd_swizzle;
    float fp16_scale;       // FP16DEV: 2^k
    float fp16_iscale;      // 2^-k
    int32_t max_steps;      // shapes taking several steps per launch: steps this launch takes
};

// Host-side launchers (return hipError_t of the launch).
int d2q9_variant_count(int coll);
const char *d2q9_variant_name(int variant);
// Steps one launch of a single-lattice D2Q9 shape takes (1, or 2 for the
// temporally blocked shapes; StepArgs::max_steps = 1 makes one of those take
// a single step), and the host-side set-up a shape needs before its first
// launch (call outside stream capture).
int d2q9_variant_steps(int coll, int variant);
hipError_t prepare_d2q9_variant(int st, int coll, int variant);
hipError_t launch_d2q9_step(int storage, int coll, int variant, const void *src, void *dst,
                            const StepArgs &a, hipStream_t s);
hipError_t launch_d2q9_batch_step(int storage, int coll, int variant, const void *src, void *dst,
                                  const StepArgs &a, hipStream_t s);
int d1q3_variant_count();
const char *d1q3_variant_name(int variant);
int d1q3_variant_steps(int variant);  // steps one launch takes at most (K-step shapes; StepArgs::max_steps sets fewer)
hipError_t prepare_d1q3_variant(int st, int batch, int variant);  // host-side set-up before the first launch
hipError_t launch_d1q3_step(int storage, int variant, const void *src, void *dst, const StepArgs &a,
                            hipStream_t s);
hipError_t launch_d1q3_batch_step(int storage, int variant, const void *src, void *dst,
                                  const StepArgs &a, hipStream_t s);
// Batch of small D2Q9 lattices resident in LDS: one workgroup per instance
// (a.ntiles = instances) runs nsteps steps in one launch; dst receives the
// final state (it may equal src).
hipError_t launch_d2q9_lds(int storage, int coll, const void *src, void *dst, const StepArgs &a, int nsteps,
                           int block, size_t smem_bytes, hipStream_t s);
// Batched shapes: count (MinxEnt4 D2Q9 batches also have two-step shapes),
// steps per launch, nodes per tile of the tile table (negative for the 2D
// tiles of a two-step shape: -(width * 4096 + rows)), name, and the
// host-side set-up before a shape's first launch.
int batch_variant_count(int lattice, int coll);
int batch_variant_steps(int lattice, int variant);
int batch_tile_nodes(int lattice, int variant);
const char *batch_variant_name(int lattice, int variant);
hipError_t prepare_batch_variant(int st, int coll, int variant);

// Set the state of one instance: pre-shifted equilibrium of FP64 fields
// (d_rho, d_ux, d_uy: nx*ny device doubles) or of FP64 populations (d_f:
// b planes of nx*ny device doubles).
hipError_t launch_init(int lattice, int storage, const Inst &in, int bc, const double *d_rho,
                       const double *d_ux, const double *d_uy, const double *d_f, void *buf,
                       float fp16_scale, hipStream_t s);
// Gather the pre-collision populations of one instance and write either its
// moments (d_rho, d_ux, d_uy) or the populations (d_f), as doubles.
hipError_t launch_gather(int lattice, int storage, const Inst &in, int bc, const void *buf,
                         double *d_rho, double *d_ux, double *d_uy, double *d_f, float fp16_iscale,
                         hipStream_t s);

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_add_step_base(int64_t *base, int64_t n, hipStream_t s);
hipError_t launch_set_step_base(int64_t *base, int64_t v, hipStream_t s);
hipError_t launch_clear_status(DevStatus *st, int n, hipStream_t s);

}  // namespace lbm
