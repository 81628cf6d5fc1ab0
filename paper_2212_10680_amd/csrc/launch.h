// Host-side launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace fl {

struct LaunchCfg {
    int lattice;    // 0 D2Q9, 1 D3Q19
    int nc;         // components
    int precision;  // 0 FP64, 1 FP32 populations
    bool mrt;
    hipStream_t stream;
    int block_k1 = 128;     // threads per block of the moments/EOS kernel
    int block_k2 = 128;     // threads per block of the collide/stream kernel
    bool xcd_remap = true;  // XCD-contiguous block order
    bool xcd_remap_k2 = true;  // the same for the plain collide/stream kernel
    bool nt_store = false;  // non-temporal population stores
    int serve_block = 512;  // threads per request in the batched server (256, 512, 1024)
    int serve_cap = -1;     // most workgroups advanced per tick, oldest request first
                            // (-1: as many as the device holds at once, 0: all running)
    int serve_group = 3584; // nodes per workgroup at which a request is split over several
                            // workgroups of one XCD (0: one workgroup per request)
    bool fused = false;     // one-launch step (fl_set_tuning "fused=1") when the lattice allows it
    bool zmarch = false;    // z-marching collide/stream kernel where zmarch_fits() (set per solver)
    bool reverse_k2 = false;  // collide/stream sweeps the nodes last to first (set per solver)
    bool slab_order = false;  // y-major row order inside per-XCD z-slabs (fl_set_tuning "order=1")
    int zlen = 16;          // planes per workgroup of the z-marching kernel
    int zorder = 0;         // block order of the z-marching kernels: 0 XCD-contiguous chunks,
                            // 1 XCD y-bands (zmarch_tile_of_block)
    bool csplit = true;     // isotropic z-marching kernel with N_c = 3: one component per
                            // 256-thread group (fl_set_tuning "csplit=0": one thread per node)
    int bands = 0;          // XCD-band order of the plain collide pass (band_node): row bands, a
                            // multiple of 8; 0 = off
    int bands_lap = 0;      // the same for the interface-Laplacian pass
    bool mpair = true;      // moments pass with two consecutive nodes per thread where it
                            // applies (k_moments_eos_pair; fl_set_tuning "mpair=0": one)
};

hipError_t launch_moments_eos(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                              double* rt, double* lnf, int* err);
// Isotropic stencils only: -lap(phi) at every node into lnf + (N_c + 1) N,
// from phi at lnf + N_c N (written by launch_moments_eos).
hipError_t launch_interface_lap(const LaunchCfg& lc, const KParams& kp, double* lnf);
// fsum_in/fsum_out: force history (population precision), previous and this step
hipError_t launch_collide_stream(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn,
                                 const float* rref, const double* rt, const double* lnf, const void* fsum_in,
                                 void* fsum_out);

// Geometry of the fused one-launch step (see k_fused_step; D3Q19 only).
struct FusedCfg {
    int tpp;            // 256-node tiles of one XCD's band of an A-plane
    int cstride;        // counters per XCD (>= nz + 2)
    unsigned target;    // counter value of a complete A-plane in this launch
    int spin_limit;     // bound on every wait loop
};
enum { kErrDomain = 1, kErrXcd = 4, kErrWait = 8 };
hipError_t launch_fused_step(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn, const float* rref,
                             double* rt, double* lnf, const void* fsum_in, void* fsum_out, unsigned* counters,
                             int* err, const FusedCfg& fc);
hipError_t launch_xcd_ids(int* out, int nblocks, hipStream_t stream);
// z-marching form of launch_collide_stream: D3Q19, N_c <= 3, nx % 64 == 0,
// ny % 4 == 0 (zmarch_fits); hipErrorInvalidValue otherwise.
bool zmarch_fits(int lattice, int nc, int nx, int ny);
hipError_t launch_collide_zmarch(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn,
                                 const float* rref, const double* rt, const double* lnf, const void* fsum_in,
                                 void* fsum_out);
// The same with the isotropic stencils (kp.iso): -lap(phi) is computed from
// phi inside the pass, so no Laplacian pass runs before it; also needs nz >= 2.
hipError_t launch_collide_zmarch_iso(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn,
                                     const float* rref, const double* rt, const double* lnf, const void* fsum_in,
                                     void* fsum_out);
hipError_t launch_init(const LaunchCfg& lc, const KParams& kp, const double* rho_molar, const double* u,
                       void* g, float* rref, void* fsum);
hipError_t launch_fields(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                         const void* fsum, double* rho_molar, double* u, double* p, double* lnf);
hipError_t launch_export_pops(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                              double* out);
// Deterministic reduction: out[0..nc) = sum_x rho_i, out[nc..2nc) = max |rho_i - snap_i|
// (snap updated; zero when snap is null), out[2nc..3nc) = max rho_i.
hipError_t launch_reduce(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                         double* snap, double* partial, double* out);
int reduce_blocks(int N);
hipError_t launch_snapshot(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref, double* snap);

// One in-flight request of the batched server (device copy updated each tick).
struct SlotDesc {
    int nx, ny, nz, N;
    long long off_pop[2];     // byte offsets into the pool
    long long off_rt, off_lnf, off_fsum, off_rref, off_snap;
    long long steps;          // steps done
    long long max_steps;
    long long check_every;
    double tol;
    double residual;
    int cur;                  // population buffer holding the current state
    int status;               // kSlotRunning, kSlotConverged, kSlotMaxSteps, kSlotNumeric
    int groups;               // workgroups advancing this request in the tick (1..kMaxGroup)
    int pad;
};
enum { kSlotRunning = 0, kSlotConverged = 1, kSlotMaxSteps = 2, kSlotNumeric = 3 };

// Workgroups of one request share this block of device memory during a tick
// (zeroed before it): barrier arrivals, the time-slice decision of workgroup
// 0, a numeric-failure flag, and each workgroup's residual maxima.
constexpr int kMaxGroup = 8;
struct GroupSync {
    unsigned count;
    int go;
    int bad;
    int pad;
    double part[kMaxGroup][2 * kMaxComp];
};
// Block b of a tick advances request table[b].x as its workgroup table[b].y
// (table[b].x < 0: the block has no work).

// Workgroups of the batched-server kernel that the device holds at once.
hipError_t serve_resident_blocks(const LaunchCfg& lc, int* blocks);
// Advance every request of descs by up to `steps` steps with `nblocks`
// workgroups mapped by table (the groups[] workgroups of a request on one
// XCD, all resident at once), each request stopping early once clock_budget
// ticks of the device wall clock have passed (<= 0: no limit); descs is
// updated in place, sync holds one GroupSync per request.
hipError_t launch_serve_tick(const LaunchCfg& lc, const KParams& kp, char* pool, SlotDesc* descs,
                             const int2* table, int nblocks, GroupSync* sync, long long steps,
                             long long clock_budget);

}  // namespace fl
