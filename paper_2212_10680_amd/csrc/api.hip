// C ABI of the fugacity-based LBM solver (see include/fuglbm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fuglbm.h"
#include "device.h"
#include "launch.h"

using fl::KParams;
using fl::LaunchCfg;

struct fl_solver {
    fl_params prm;                         // copy (pointers re-targeted below)
    std::vector<fl_component> comp;
    std::vector<double> kij;
    double mrt[4];
    KParams kp;
    LaunchCfg lc;
    int D, Q, nc;
    size_t N;
    size_t pop_elem;                       // bytes per population value
    // device buffers
    void* mem = nullptr;
    bool own_mem = false;
    void* pop[2] = {nullptr, nullptr};
    int cur = 0;
    double* rt = nullptr;
    double* lnf = nullptr;
    void* fsum[2] = {nullptr, nullptr};    // force history (population precision), double-buffered
    int fcur = 0;
    unsigned* counters = nullptr;          // per-XCD plane counters of the fused step
    bool fused = false;                    // one-launch step in use
    bool zmarch = false;                   // z-marching collide/stream kernel in use
    fl::FusedCfg fc{};
    unsigned fused_launches = 0;
    float* rref = nullptr;
    double* snap = nullptr;
    double* out = nullptr;                 // (D + 1) * N scratch for field export
    double* partial = nullptr;
    double* red = nullptr;                 // 3*nc reduction results
    int* err = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int* h_err = nullptr;                  // pinned host mirrors
    double* h_red = nullptr;
    long steps = 0;
    bool snap_valid = false;
    std::vector<hipEvent_t> timing_events;  // fl_step_timed's, created on its first call
    std::string last_error;
};

namespace {

constexpr double kOmega[3][2] = {{0.457235529, 0.077796074},   // PR (App. C.1)
                                 {0.4274802, 0.08664035},      // SRK
                                 {27.0 / 64.0, 1.0 / 8.0}};    // vdW

int fail(fl_solver* s, int code, const std::string& msg) {
    if (s) s->last_error = msg;
    return code;
}

int hip_fail(fl_solver* s, hipError_t e, const char* where) {
    return fail(s, FL_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(s, expr)                                          \
    do {                                                          \
        hipError_t _e = (expr);                                   \
        if (_e != hipSuccess) return hip_fail((s), _e, #expr);    \
    } while (0)

int lattice_dims(int lattice, int* D, int* Q) {
    if (lattice == FL_D2Q9) { *D = 2; *Q = 9; return 0; }
    if (lattice == FL_D3Q19) { *D = 3; *Q = 19; return 0; }
    return -1;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t pop, rt, lnf, fsum, rref, snap, out, partial, red, err, counters, total;
};

Layout layout_for(const fl_params* p) {
    int D, Q;
    lattice_dims(p->lattice, &D, &Q);
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const size_t nc = p->ncomp;
    const size_t es = p->precision == FL_FP64 ? 8 : 4;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.pop = take(2 * nc * Q * N * es);
    L.rt = take(nc * N * 8);
    // ln f_i, then the interface field phi (and -lap(phi) with the isotropic stencils)
    L.lnf = take((nc + 1 + (p->stencil == FL_STENCIL_ISOTROPIC ? 1 : 0)) * N * 8);
    L.fsum = take(2 * (size_t)D * N * es);
    L.rref = take(p->precision == FL_FP64 ? 0 : nc * N * 4);
    L.snap = take(nc * N * 8);
    L.out = take((size_t)(D + 1) * N * 8);
    L.partial = take((size_t)fl::reduce_blocks((int)N) * 3 * nc * 8);
    L.red = take(3 * nc * 8);
    L.err = take(256);
    L.counters = take((size_t)8 * (p->nz + 8) * sizeof(unsigned));
    L.total = off;
    return L;
}

// Host-side EOS constants (App. C.1): a_i, b_i, alpha_i(T), (a alpha)_ij.
void eos_constants(const fl_solver* s, KParams* kp) {
    const fl_params& p = s->prm;
    const int nc = p.ncomp;
    const double Oa = kOmega[p.eos][0], Ob = kOmega[p.eos][1];
    double aa[fl::kMaxComp];
    for (int i = 0; i < nc; ++i) {
        const fl_component& c = s->comp[i];
        const double a = Oa * p.R * p.R * c.Tc * c.Tc / c.Pc;
        kp->b[i] = Ob * p.R * c.Tc / c.Pc;
        const double tr = p.T / c.Tc;
        double alpha = 1.0;
        if (p.eos == FL_EOS_PR) {
            const double w = c.omega;
            const double m = (w <= 0.49) ? 0.374640 + 1.54226 * w - 0.26992 * w * w
                                         : 0.379642 + 1.48503 * w - 0.164423 * w * w + 0.016666 * w * w * w;
            alpha = (1.0 + m * (1.0 - std::sqrt(tr))) * (1.0 + m * (1.0 - std::sqrt(tr)));
        } else if (p.eos == FL_EOS_SRK) {
            const double w = c.omega;
            const double m = 0.48 + 1.574 * w - 0.176 * w * w;
            alpha = (1.0 + m * (1.0 - std::sqrt(tr))) * (1.0 + m * (1.0 - std::sqrt(tr)));
        }
        aa[i] = a * alpha;
        kp->M[i] = c.M;
    }
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
            kp->aa[i * nc + j] = std::sqrt(aa[i] * aa[j]) * (1.0 - s->kij[i * nc + j]);
            kp->kap[i * nc + j] = std::sqrt(s->comp[i].kappa * s->comp[j].kappa);
        }
    for (int i = 0; i < nc; ++i) kp->sk[i] = std::sqrt(s->comp[i].kappa);
}

// Host copy of the device EOS domain test for fl_set_state.
bool host_in_domain(const KParams& kp, int nc, const double* rt) {
    double r = 0.0;
    for (int i = 0; i < nc; ++i) {
        if (!(rt[i] > 0.0) || !std::isfinite(rt[i])) return false;
        r += rt[i];
    }
    double bm = 0.0;
    for (int i = 0; i < nc; ++i) bm += rt[i] / r * kp.b[i];
    return bm * r < 1.0;
}

// Measured default launch choices for a solver's lattice (kernel variants,
// block sizes and visiting orders; none of them changes a result bit).
void default_launch(fl_solver* s) {
    const fl_params& p = s->prm;
    LaunchCfg& lc = s->lc;
    lc.block_k1 = 128;
    lc.block_k2 = 128;
    lc.xcd_remap = true;
    lc.xcd_remap_k2 = true;
    lc.nt_store = false;
    lc.fused = false;
    lc.slab_order = false;
    lc.zlen = 16;
    lc.csplit = true;
    lc.mpair = true;
    lc.zorder = 0;
    lc.bands = 0;
    lc.bands_lap = 0;
    // The collide/stream pass sweeps the nodes in the opposite order to the
    // moments pass when one population buffer is within a few times the 256 MB
    // memory-side cache: each pass then starts on the lines the other touched
    // last.  Larger lattices gain nothing from it.
    lc.reverse_k2 = (double)s->nc * s->Q * s->N * s->pop_elem <= 1073741824.0;
    // The z-marching collide kernel (stencil fields staged through LDS) is the
    // faster one with one or two components; with three and the axis stencils
    // its registers cost more than the re-reads it saves (measured on the
    // 256^3 ternary lattice).  With the isotropic stencils the plain kernel's
    // 18-neighbour gathers of seven FP64 fields set its time, and the
    // z-marching form (which also computes -lap(phi) itself) is used.
    lc.zmarch = p.ncomp <= 2 || p.stencil == FL_STENCIL_ISOTROPIC;
    // Plain collide kernel block size: 128 threads with the interleaved layout
    // (N_c <= 2), 256 with the component-major one, whose N_c * Q streams of
    // 4 B per node read and write in longer runs per block (measured:
    // 256^3 ternary 2.32 -> 2.15 ms, 128^3 binary 0.169 -> 0.178 ms the other way).
    lc.block_k2 = p.ncomp >= 3 ? 256 : 128;
    // ... and takes its blocks in plain order there (2.15 -> 2.09 ms on the
    // 256^3 ternary lattice; the moments pass keeps the XCD-contiguous order).
    lc.xcd_remap_k2 = p.ncomp <= 2;
    // With the isotropic stencils and N_c >= 3 the collide pass is bound by its
    // re-reads of the stencil fields rather than by the population streams:
    // 64-thread blocks in XCD-contiguous order are the fastest there (256^3
    // ternary: 3.85 ms at 256, 3.40 at 128, 3.13 at 64, 3.07 with the XCD
    // order; the binary lattice stays best at 128).
    if (p.stencil == FL_STENCIL_ISOTROPIC && p.ncomp >= 3) {
        lc.block_k2 = 64;
        lc.xcd_remap_k2 = true;
        // The z-marching form there gives each component its own 256 threads
        // (three waves per SIMD instead of one: the same time, 2.51 ms on the
        // 256^3 ternary lattice, with its fills where the other form has them;
        // 2.34 ms with the fills after the pushes), takes its workgroups in
        // XCD y-bands, so that all XCDs march through the same planes at once
        // (2.60 -> 2.51 ms against XCD-contiguous chunks), and runs 32 planes
        // per workgroup (2.34 -> 2.31 ms; 24 planes 2.33).
        // In FP64 the split form spills (9.87 ms per step against 6.42 for the
        // plain collide kernel and the Laplacian pass), and the one-thread-per-
        // node z-march in this order takes 6.19 ms.
        lc.csplit = p.precision != FL_FP64;
        lc.zorder = 1;
        lc.zlen = 32;
        // The moments pass (no stencil, so nothing for an XCD's L2 to keep)
        // then streams best in plain block order, all XCDs in one window of
        // addresses, with 256-thread blocks: 0.963 -> 0.937 ms on the 256^3
        // ternary FP32 lattice (64: 0.974), 1.665 -> 1.578 ms in FP64.
        lc.xcd_remap = false;
        lc.block_k1 = 256;
    }
}

int xcd_placement_ok(hipStream_t stream);

// Which kernels a step launches, from the launch choices and the lattice.
void choose_paths(fl_solver* s) {
    const fl_params& p = s->prm;
    // (the isotropic z-marching kernels need two planes or more)
    s->zmarch = s->lc.zmarch && fl::zmarch_fits(p.lattice, p.ncomp, p.nx, p.ny) && (s->kp.iso == 0 || p.nz >= 2);
    // one-launch step: D3Q19, >= 8 rows per XCD (halo recompute <= 50 %), rows
    // of whole 128-byte lines of the FP64 density arrays, blocks placed on XCD b % 8
    s->fused = s->lc.fused && s->kp.iso == 0 && s->D == 3 && p.ny >= 64 && p.nx % 16 == 0 && p.nz >= 4 &&
               xcd_placement_ok(s->stream);
}

// Parses a launch-tuning spec "key=value[,key=value...]" into lc.  Solver
// keys: k1block, k2block (64..256, multiples of 64), remap, remap2, nt, fused,
// zmarch, rev, order, zorder, csplit, mpair (0/1), zlen (1..4096), bands, lapbands
// (0..1024, multiples of 8); server keys: serve (256, 512, 1024), serve_cap
// (-1..2^20), serve_group (0..2^24).  Returns false (lc unchanged) for an unknown key
// or an out-of-range value.
bool parse_tuning(LaunchCfg& lc, const char* spec, bool server) {
    LaunchCfg t = lc;
    std::string str(spec);
    size_t pos = 0;
    while (pos <= str.size()) {
        size_t comma = str.find(',', pos);
        if (comma == std::string::npos) comma = str.size();
        const std::string item = str.substr(pos, comma - pos);
        pos = comma + 1;
        if (item.empty()) continue;
        const size_t eq = item.find('=');
        if (eq == std::string::npos) return false;
        const std::string key = item.substr(0, eq);
        char* endp = nullptr;
        const long v = std::strtol(item.c_str() + eq + 1, &endp, 10);
        if (endp == item.c_str() + eq + 1 || *endp != '\0') return false;
        const bool flag = v == 0 || v == 1;
        if (!server && (key == "k1block" || key == "k2block")) {
            if (v < 64 || v > 256 || v % 64) return false;
            (key == "k1block" ? t.block_k1 : t.block_k2) = (int)v;
        } else if (!server && key == "remap" && flag) {
            t.xcd_remap = t.xcd_remap_k2 = v != 0;
        } else if (!server && key == "remap2" && flag) {
            t.xcd_remap_k2 = v != 0;
        } else if (!server && key == "nt" && flag) {
            t.nt_store = v != 0;
        } else if (!server && key == "fused" && flag) {
            t.fused = v != 0;
        } else if (!server && key == "zmarch" && flag) {
            t.zmarch = v != 0;
        } else if (!server && key == "rev" && flag) {
            t.reverse_k2 = v != 0;
        } else if (!server && key == "order" && flag) {
            t.slab_order = v != 0;
        } else if (!server && key == "zorder" && flag) {
            t.zorder = (int)v;
        } else if (!server && key == "csplit" && flag) {
            t.csplit = v != 0;
        } else if (!server && key == "mpair" && flag) {
            t.mpair = v != 0;
        } else if (!server && key == "zlen" && v >= 1 && v <= 4096) {
            t.zlen = (int)v;
        } else if (!server && (key == "bands" || key == "lapbands") && v >= 0 && v <= 1024 && v % 8 == 0) {
            (key == "bands" ? t.bands : t.bands_lap) = (int)v;
        } else if (server && key == "serve" && (v == 256 || v == 512 || v == 1024)) {
            t.serve_block = (int)v;
        } else if (server && key == "serve_cap" && v >= -1 && v <= 1 << 20) {
            t.serve_cap = (int)v;
        } else if (server && key == "serve_group" && v >= 0 && v <= 1 << 24) {
            t.serve_group = (int)v;
        } else {
            return false;
        }
    }
    lc = t;
    return true;
}

int setup(fl_solver* s, const fl_params* p) {
    s->prm = *p;
    s->comp.assign(p->comp, p->comp + p->ncomp);
    s->kij.assign((size_t)p->ncomp * p->ncomp, 0.0);
    if (p->kij) std::memcpy(s->kij.data(), p->kij, sizeof(double) * p->ncomp * p->ncomp);
    s->prm.comp = s->comp.data();
    s->prm.kij = s->kij.data();
    if (p->mrt_rates) {
        std::memcpy(s->mrt, p->mrt_rates, sizeof(s->mrt));
    } else {
        s->mrt[0] = 1.0 / p->tau;
        s->mrt[1] = 1.0 / p->tau;
        s->mrt[2] = 1.0;
        s->mrt[3] = 1.0;
    }
    s->prm.mrt_rates = s->mrt;
    lattice_dims(p->lattice, &s->D, &s->Q);
    s->nc = p->ncomp;
    s->N = (size_t)p->nx * p->ny * p->nz;
    s->pop_elem = p->precision == FL_FP64 ? 8 : 4;
    KParams& kp = s->kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.nx = p->nx;
    kp.ny = p->ny;
    kp.nz = p->nz;
    kp.N = (int)s->N;
    kp.eos = p->eos;
    kp.force_level = p->force_time_level;
    kp.standard = p->force_model == FL_FORCE_STANDARD ? 1 : 0;
    kp.iso = p->stencil == FL_STENCIL_ISOTROPIC ? 1 : 0;
    kp.RT = p->R * p->T;
    kp.lnRT = std::log(kp.RT);
    kp.omega = 1.0 / p->tau;
    kp.cF = 1.0 - 1.0 / (2.0 * p->tau);
    kp.s_j = s->mrt[0];
    kp.s_nu = s->mrt[1];
    kp.s_e = s->mrt[2];
    kp.s_g = s->mrt[3];
    {
        // squared norms of the group rows of the orthogonal moment bases
        // (Lallemand-Luo D2Q9, d'Humieres D3Q19), in the order of collide()
        const double dj = kp.s_j - kp.s_g, dn = kp.s_nu - kp.s_g, de = kp.s_e - kp.s_g;
        if (p->lattice == FL_D2Q9) {
            const double f[5] = {dj / 6, dj / 6, dn / 4, dn / 4, de / 36};
            for (int k = 0; k < 5; ++k) kp.mrt_f[k] = f[k];
        } else {
            const double f[9] = {dj / 10, dj / 10, dj / 10, dn / 36, dn / 12, dn / 4, dn / 4, dn / 4, de / 2394};
            for (int k = 0; k < 9; ++k) kp.mrt_f[k] = f[k];
        }
    }
    eos_constants(s, &kp);
    s->lc.lattice = p->lattice;
    s->lc.nc = p->ncomp;
    s->lc.precision = p->precision;
    s->lc.mrt = p->collision == FL_MRT;
    {
        // fused-step geometry: each XCD owns ny/8 (+1) rows plus 4 halo rows
        const int rowsA = (p->ny + 7) / 8 + 4;
        s->fc.tpp = (rowsA * p->nx + 255) / 256;
        s->fc.cstride = p->nz + 8;
        s->fc.target = 0;
        s->fc.spin_limit = 1 << 20;   // about 60 ms of s_sleep per wait
    }
    default_launch(s);
    choose_paths(s);
    return FL_OK;
}

int carve(fl_solver* s, void* base) {
    const Layout L = layout_for(&s->prm);
    char* b = (char*)base;
    const size_t half = s->nc * s->Q * s->N * s->pop_elem;
    s->pop[0] = b + L.pop;
    s->pop[1] = b + L.pop + half;
    s->rt = (double*)(b + L.rt);
    s->lnf = (double*)(b + L.lnf);
    s->fsum[0] = (void*)(b + L.fsum);
    s->fsum[1] = (void*)(b + L.fsum + (size_t)s->D * s->N * s->pop_elem);
    s->counters = (unsigned*)(b + L.counters);
    s->rref = s->prm.precision == FL_FP64 ? nullptr : (float*)(b + L.rref);
    s->snap = (double*)(b + L.snap);
    s->out = (double*)(b + L.out);
    s->partial = (double*)(b + L.partial);
    s->red = (double*)(b + L.red);
    s->err = (int*)(b + L.err);
    choose_paths(s);
    HIP_TRY(s, hipHostMalloc((void**)&s->h_err, sizeof(int) * 4, hipHostMallocDefault));
    HIP_TRY(s, hipHostMalloc((void**)&s->h_red, sizeof(double) * 3 * fl::kMaxComp, hipHostMallocDefault));
    HIP_TRY(s, hipMemsetAsync(s->err, 0, 256, s->stream));
    HIP_TRY(s, hipMemsetAsync(s->pop[0], 0, 2 * half, s->stream));
    HIP_TRY(s, hipMemsetAsync(s->fsum[0], 0, 2 * (size_t)s->D * s->N * s->pop_elem, s->stream));
    HIP_TRY(s, hipMemsetAsync(s->counters, 0, (size_t)8 * s->fc.cstride * sizeof(unsigned), s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return FL_OK;
}

// Read and clear the device error flag (synchronises the stream).
int check_err(fl_solver* s) {
    HIP_TRY(s, hipMemcpyAsync(s->h_err, s->err, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    if (*s->h_err) {
        const int flags = *s->h_err;
        HIP_TRY(s, hipMemsetAsync(s->err, 0, sizeof(int), s->stream));
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        if (flags & (fl::kErrXcd | fl::kErrWait)) {
            s->fused = false;  // later steps use the two-kernel path
            return fail(s, FL_EDEVICE, (flags & fl::kErrXcd) ? "fused step: a block ran on an unexpected XCD"
                                                              : "fused step: a dependency wait timed out");
        }
        return fail(s, FL_ENUMERIC, "a node left the EOS domain (rho~_i <= 0, rho~ b_m >= 1 or non-finite)");
    }
    return FL_OK;
}

int one_step(fl_solver* s, hipEvent_t* ev) {
    void* g = s->pop[s->cur];
    void* gn = s->pop[1 - s->cur];
    LaunchCfg lc = s->lc;
    lc.stream = s->stream;
    if (ev) HIP_TRY(s, hipEventRecord(ev[0], s->stream));
    if (s->fused) {
        fl::FusedCfg fc = s->fc;
        fc.target = (unsigned)fc.tpp * (s->fused_launches + 1u);
        HIP_TRY(s, fl::launch_fused_step(lc, s->kp, g, gn, s->rref, s->rt, s->lnf, s->fsum[s->fcur],
                                         s->fsum[1 - s->fcur], s->counters, s->err, fc));
        s->fused_launches += 1;
        if (ev) HIP_TRY(s, hipEventRecord(ev[1], s->stream));
    } else {
        HIP_TRY(s, fl::launch_moments_eos(lc, s->kp, g, s->rref, s->rt, s->lnf, s->err));
        if (ev) HIP_TRY(s, hipEventRecord(ev[1], s->stream));
        // the z-marching form computes -lap(phi) itself; the plain kernel reads
        // it from a pass of its own
        if (s->kp.iso && !s->zmarch) {
            HIP_TRY(s, fl::launch_interface_lap(lc, s->kp, s->lnf));
            if (ev) HIP_TRY(s, hipEventRecord(ev[2], s->stream));
        }
        if (s->zmarch && s->kp.iso)
            HIP_TRY(s, fl::launch_collide_zmarch_iso(lc, s->kp, g, gn, s->rref, s->rt, s->lnf, s->fsum[s->fcur],
                                                     s->fsum[1 - s->fcur]));
        else if (s->zmarch)
            HIP_TRY(s, fl::launch_collide_zmarch(lc, s->kp, g, gn, s->rref, s->rt, s->lnf, s->fsum[s->fcur],
                                                 s->fsum[1 - s->fcur]));
        else
            HIP_TRY(s, fl::launch_collide_stream(lc, s->kp, g, gn, s->rref, s->rt, s->lnf, s->fsum[s->fcur],
                                                 s->fsum[1 - s->fcur]));
        if (ev) HIP_TRY(s, hipEventRecord(ev[3], s->stream));
    }
    s->cur = 1 - s->cur;
    s->fcur = 1 - s->fcur;
    s->steps += 1;
    return FL_OK;
}

// Blocks of one launch run on XCD (block index % 8): checked once per process.
int xcd_placement_ok(hipStream_t stream) {
    static int placement = -1;
    if (placement >= 0) return placement;
    const int nb = 4096;
    int* d = nullptr;
    std::vector<int> h(nb, -1);
    placement = 0;
    if (hipMalloc(&d, nb * sizeof(int)) != hipSuccess) { (void)hipGetLastError(); return placement; }
    if (fl::launch_xcd_ids(d, nb, stream) == hipSuccess &&
        hipMemcpyAsync(h.data(), d, nb * sizeof(int), hipMemcpyDeviceToHost, stream) == hipSuccess &&
        hipStreamSynchronize(stream) == hipSuccess) {
        placement = 1;
        for (int b = 0; b < nb; ++b)
            if (h[b] != b % 8) placement = 0;
    }
    (void)hipFree(d);
    (void)hipGetLastError();
    return placement;
}

int reduce(fl_solver* s, bool with_snap) {
    LaunchCfg lc = s->lc;
    lc.stream = s->stream;
    HIP_TRY(s, fl::launch_reduce(lc, s->kp, s->pop[s->cur], s->rref, with_snap ? s->snap : nullptr,
                                 s->partial, s->red));
    HIP_TRY(s, hipMemcpyAsync(s->h_red, s->red, sizeof(double) * 3 * s->nc, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return FL_OK;
}

}  // namespace

extern "C" {

const char* fl_status_string(int st) {
    switch (st) {
        case FL_OK: return "ok";
        case FL_EINVAL: return "invalid argument";
        case FL_EDOMAIN: return "state outside the EOS domain";
        case FL_ENOMEM: return "out of memory";
        case FL_EDEVICE: return "HIP device error";
        case FL_ENUMERIC: return "numerical failure during stepping";
        case FL_ENOTCONV: return "not converged";
        case FL_EAGAIN: return "try again";
        default: return "unknown status";
    }
}

int fl_validate(const fl_params* p) {
    if (!p || !p->comp) return FL_EINVAL;
    if (p->ncomp < 1 || p->ncomp > FL_MAX_COMP) return FL_EINVAL;
    int D, Q;
    if (lattice_dims(p->lattice, &D, &Q)) return FL_EINVAL;
    if (p->eos < FL_EOS_PR || p->eos > FL_EOS_VDW) return FL_EINVAL;
    if (p->collision != FL_BGK && p->collision != FL_MRT) return FL_EINVAL;
    if (p->precision != FL_FP64 && p->precision != FL_FP32POP_FP64EOS) return FL_EINVAL;
    if (p->force_time_level != 0 && p->force_time_level != 1) return FL_EINVAL;
    if (p->force_model != FL_FORCE_WB && p->force_model != FL_FORCE_STANDARD) return FL_EINVAL;
    if (p->force_model == FL_FORCE_STANDARD && p->precision != FL_FP64) return FL_EINVAL;
    if (p->stencil != FL_STENCIL_AXIS && p->stencil != FL_STENCIL_ISOTROPIC) return FL_EINVAL;
    if (!(p->tau > 0.5) || !(p->T > 0.0) || !(p->R > 0.0)) return FL_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return FL_EINVAL;
    if (D == 2 && p->nz != 1) return FL_EINVAL;
    const double N = (double)p->nx * p->ny * p->nz;
    // byte offsets within one array stay below 2^32: the FP64 fields (8 B per
    // node and component), one direction's populations (N_c per node) and the
    // force history (D per node)
    if (N >= 536870912.0) return FL_EINVAL;  // 2^29
    const double elem = p->precision == FL_FP64 ? 8.0 : 4.0;
    if (N * p->ncomp * elem >= 4294967296.0) return FL_EINVAL;
    // ... and the force history fsum[n][k] (D values per node)
    if (N * D * elem >= 4294967296.0) return FL_EINVAL;
    for (int i = 0; i < p->ncomp; ++i) {
        const fl_component& c = p->comp[i];
        if (!(c.Tc > 0) || !(c.Pc > 0) || !(c.M > 0) || !(c.kappa >= 0) || !std::isfinite(c.omega))
            return FL_EINVAL;
    }
    if (p->kij)
        for (int i = 0; i < p->ncomp; ++i)
            for (int j = 0; j < p->ncomp; ++j) {
                const double a = p->kij[i * p->ncomp + j], b = p->kij[j * p->ncomp + i];
                if (!std::isfinite(a) || a != b || (i == j && a != 0.0)) return FL_EINVAL;
            }
    if (p->collision == FL_MRT && p->mrt_rates)
        for (int k = 0; k < 4; ++k)
            if (!(p->mrt_rates[k] > 0.0 && p->mrt_rates[k] < 2.0)) return FL_EINVAL;
    return FL_OK;
}

int fl_set_tuning(fl_solver* s, const char* spec) {
    if (!s) return FL_EINVAL;
    const LaunchCfg saved = s->lc;
    default_launch(s);
    if (spec && !parse_tuning(s->lc, spec, false)) {
        s->lc = saved;
        return fail(s, FL_EINVAL, std::string("unknown tuning key or value in \"") + spec + "\"");
    }
    // the one-launch step counts its launches from zeroed plane counters
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    HIP_TRY(s, hipMemsetAsync(s->counters, 0, (size_t)8 * s->fc.cstride * sizeof(unsigned), s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->fused_launches = 0;
    choose_paths(s);
    return FL_OK;
}

int fl_required_bytes(const fl_params* p, size_t* bytes) {
    const int v = fl_validate(p);
    if (v != FL_OK) return v;
    if (!bytes) return FL_EINVAL;
    *bytes = layout_for(p).total;
    return FL_OK;
}

static int create_common(const fl_params* p, void* mem, size_t bytes, void* stream, bool own, fl_solver** out) {
    if (!out) return FL_EINVAL;
    *out = nullptr;
    const int v = fl_validate(p);
    if (v != FL_OK) return v;
    fl_solver* s = new (std::nothrow) fl_solver();
    if (!s) return FL_ENOMEM;
    setup(s, p);
    const size_t need = layout_for(&s->prm).total;
    if (own) {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete s; return FL_EDEVICE; }
        s->own_stream = true;
        e = hipMalloc(&s->mem, need);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(s->stream);
            delete s;
            (void)hipGetLastError();
            return FL_ENOMEM;
        }
        s->own_mem = true;
    } else {
        if (!mem || bytes < need || ((uintptr_t)mem & 255)) { delete s; return FL_ENOMEM; }
        s->mem = mem;
        s->stream = (hipStream_t)stream;
    }
    const int c = carve(s, s->mem);
    if (c != FL_OK) { fl_destroy(s); return c; }
    *out = s;
    return FL_OK;
}

int fl_create(const fl_params* p, fl_solver** out) { return create_common(p, nullptr, 0, nullptr, true, out); }

int fl_create_ext(const fl_params* p, void* device_mem, size_t bytes, void* hip_stream, fl_solver** out) {
    return create_common(p, device_mem, bytes, hip_stream, false, out);
}

void fl_destroy(fl_solver* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (hipEvent_t e : s->timing_events)
        if (e) (void)hipEventDestroy(e);
    if (s->own_mem && s->mem) (void)hipFree(s->mem);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    if (s->h_err) (void)hipHostFree(s->h_err);
    if (s->h_red) (void)hipHostFree(s->h_red);
    delete s;
}

const char* fl_last_error(const fl_solver* s) { return s ? s->last_error.c_str() : "null solver"; }

int fl_lattice_table(int lattice, int* q, int* e, double* w) {
    int D, Q;
    if (lattice_dims(lattice, &D, &Q)) return FL_EINVAL;
    if (q) *q = Q;
    for (int a = 0; a < Q; ++a) {
        int ex, ey, ez;
        double wa;
        if (lattice == FL_D2Q9) {
            ex = fl::Lat<0>::ex[a]; ey = fl::Lat<0>::ey[a]; ez = 0; wa = fl::Lat<0>::w[a];
        } else {
            ex = fl::Lat<1>::ex[a]; ey = fl::Lat<1>::ey[a]; ez = fl::Lat<1>::ez[a]; wa = fl::Lat<1>::w[a];
        }
        if (e) { e[3 * a] = ex; e[3 * a + 1] = ey; e[3 * a + 2] = ez; }
        if (w) w[a] = wa;
    }
    return FL_OK;
}

int fl_set_state(fl_solver* s, const double* rho_molar, const double* u) {
    if (!s || !rho_molar) return FL_EINVAL;
    const size_t N = s->N;
    const int nc = s->nc;
    std::vector<double> node(nc);
    for (size_t n = 0; n < N; ++n) {
        for (int c = 0; c < nc; ++c) node[c] = rho_molar[(size_t)c * N + n];
        if (!host_in_domain(s->kp, nc, node.data()))
            return fail(s, FL_EDOMAIN, "initial state outside the EOS domain at node " + std::to_string(n));
        if (u)
            for (int k = 0; k < s->D; ++k)
                if (!std::isfinite(u[(size_t)k * N + n])) return fail(s, FL_EDOMAIN, "non-finite velocity");
    }
    // stage densities in rt and velocity in the output scratch
    HIP_TRY(s, hipMemcpyAsync(s->rt, rho_molar, sizeof(double) * nc * N, hipMemcpyHostToDevice, s->stream));
    if (u) HIP_TRY(s, hipMemcpyAsync(s->out, u, sizeof(double) * s->D * N, hipMemcpyHostToDevice, s->stream));
    LaunchCfg lc = s->lc;
    lc.stream = s->stream;
    s->cur = 0;
    s->fcur = 0;
    s->fused_launches = 0;
    HIP_TRY(s, hipMemsetAsync(s->counters, 0, (size_t)8 * s->fc.cstride * sizeof(unsigned), s->stream));
    HIP_TRY(s, fl::launch_init(lc, s->kp, s->rt, u ? s->out : nullptr, s->pop[0], s->rref, s->fsum[0]));
    HIP_TRY(s, hipMemsetAsync(s->err, 0, sizeof(int), s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->steps = 0;
    s->snap_valid = false;
    return FL_OK;
}

int fl_step(fl_solver* s, long nsteps) {
    if (!s || nsteps < 0) return FL_EINVAL;
    for (long k = 0; k < nsteps; ++k) {
        const int r = one_step(s, nullptr);
        if (r != FL_OK) return r;
    }
    return check_err(s);
}

int fl_step_timed_every(fl_solver* s, long nsteps, long every, double* kernel_ms, const char** names,
                        int* nkernels, long* timed_steps) {
    if (!s || nsteps < 0 || every < 1 || !kernel_ms || !nkernels ||
        *nkernels < ((s->kp.iso && !s->zmarch) ? 3 : 2))
        return FL_EINVAL;
    static const char* kNames[2] = {"k_moments_eos", "k_collide_stream"};
    static const char* kFused[1] = {"k_fused_step"};
    const bool fused = s->fused;
    const bool iso = s->kp.iso != 0 && !s->zmarch;   // a Laplacian pass runs
    const long chunk = 256;
    // events are created once per solver (creating 1024 of them takes
    // milliseconds, which a timed run should not include); per timed step:
    // start, after the moments pass, after the Laplacian pass (isotropic
    // stencils), after the collide pass
    if (s->timing_events.empty()) {
        std::vector<hipEvent_t> made(4 * chunk, nullptr);
        for (auto& e : made) {
            const hipError_t c = hipEventCreate(&e);
            if (c != hipSuccess) {
                for (hipEvent_t x : made)
                    if (x) (void)hipEventDestroy(x);
                return hip_fail(s, c, "hipEventCreate");
            }
        }
        s->timing_events.swap(made);
    }
    std::vector<hipEvent_t>& ev = s->timing_events;
    double acc[3] = {0.0, 0.0, 0.0};
    long timed = 0;
    int rc = FL_OK;
    // steps in chunks of `chunk` timed ones (the event pool), then one sync
    for (long done = 0; done < nsteps && rc == FL_OK;) {
        long j = 0;
        for (; done < nsteps && j < chunk && rc == FL_OK; ++done) {
            if (done % every == 0)
                rc = one_step(s, &ev[4 * j++]);
            else
                rc = one_step(s, nullptr);
        }
        if (rc != FL_OK) break;
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) { rc = hip_fail(s, e, "hipStreamSynchronize"); break; }
        for (long k = 0; k < j; ++k) {
            hipEvent_t* e4 = &ev[4 * k];
            float a = 0.f, b = 0.f, l = 0.f;
            (void)hipEventElapsedTime(&a, e4[0], e4[1]);
            if (!fused && iso) {
                (void)hipEventElapsedTime(&l, e4[1], e4[2]);
                (void)hipEventElapsedTime(&b, e4[2], e4[3]);
            } else if (!fused) {
                (void)hipEventElapsedTime(&b, e4[1], e4[3]);
            }
            acc[0] += a;
            acc[1] += b;
            acc[2] += l;
        }
        timed += j;
    }
    if (rc != FL_OK) return rc;
    if (timed_steps) *timed_steps = timed;
    if (fused) {
        kernel_ms[0] = acc[0];
        if (names) names[0] = kFused[0];
        *nkernels = 1;
    } else {
        kernel_ms[0] = acc[0];
        kernel_ms[1] = acc[1];
        if (names) {
            names[0] = kNames[0];
            names[1] = !s->zmarch ? kNames[1]
                       : !s->kp.iso ? "k_collide_zmarch"
                       : (s->nc == 3 && s->lc.csplit) ? "k_collide_zmarch_iso_cs"
                                                       : "k_collide_zmarch_iso";
        }
        *nkernels = 2;
        if (iso) {
            kernel_ms[2] = acc[2];
            if (names) names[2] = "k_interface_lap";
            *nkernels = 3;
        }
    }
    return check_err(s);
}

int fl_step_timed(fl_solver* s, long nsteps, double* kernel_ms, const char** names, int* nkernels) {
    return fl_step_timed_every(s, nsteps, 1, kernel_ms, names, nkernels, nullptr);
}

long fl_steps_done(const fl_solver* s) { return s ? s->steps : -1; }

int fl_get_fields(fl_solver* s, double* rho_molar, double* u, double* p, double* lnf) {
    if (!s) return FL_EINVAL;
    const size_t N = s->N;
    LaunchCfg lc = s->lc;
    lc.stream = s->stream;
    // rt/lnf are rewritten by the next step's first kernel, so they can hold
    // the exported densities and ln f; out holds u then p.
    double* d_u = s->out;
    double* d_p = s->out + (size_t)s->D * N;
    HIP_TRY(s, fl::launch_fields(lc, s->kp, s->pop[s->cur], s->rref, s->fsum[s->fcur], s->rt, d_u, d_p, s->lnf));
    if (rho_molar) HIP_TRY(s, hipMemcpyAsync(rho_molar, s->rt, sizeof(double) * s->nc * N, hipMemcpyDeviceToHost, s->stream));
    if (u) HIP_TRY(s, hipMemcpyAsync(u, d_u, sizeof(double) * s->D * N, hipMemcpyDeviceToHost, s->stream));
    if (p) HIP_TRY(s, hipMemcpyAsync(p, d_p, sizeof(double) * N, hipMemcpyDeviceToHost, s->stream));
    if (lnf) HIP_TRY(s, hipMemcpyAsync(lnf, s->lnf, sizeof(double) * s->nc * N, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return FL_OK;
}

int fl_get_populations(fl_solver* s, double* g) {
    if (!s || !g) return FL_EINVAL;
    const size_t N = s->N;
    const size_t bytes = sizeof(double) * s->nc * s->Q * N;
    double* tmp = nullptr;
    HIP_TRY(s, hipMallocAsync((void**)&tmp, bytes, s->stream));
    LaunchCfg lc = s->lc;
    lc.stream = s->stream;
    hipError_t e = fl::launch_export_pops(lc, s->kp, s->pop[s->cur], s->rref, tmp);
    if (e == hipSuccess) e = hipMemcpyAsync(g, tmp, bytes, hipMemcpyDeviceToHost, s->stream);
    (void)hipFreeAsync(tmp, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "fl_get_populations");
    return FL_OK;
}

int fl_mass(fl_solver* s, double* mass) {
    if (!s || !mass) return FL_EINVAL;
    const int r = reduce(s, false);
    if (r != FL_OK) return r;
    for (int c = 0; c < s->nc; ++c) mass[c] = s->h_red[c];
    return FL_OK;
}

int fl_run_until(fl_solver* s, double tol, long check_every, long max_steps, long* steps_done, double* residual) {
    if (!s || check_every < 1 || max_steps < 0 || !(tol >= 0.0)) return FL_EINVAL;
    long done = 0;
    double res = INFINITY;
    int rc = reduce(s, true);   // snapshot of the starting densities
    if (rc != FL_OK) return rc;
    while (done < max_steps) {
        const long m = std::min(check_every, max_steps - done);
        for (long k = 0; k < m; ++k) {
            rc = one_step(s, nullptr);
            if (rc != FL_OK) return rc;
        }
        done += m;
        rc = check_err(s);
        if (rc != FL_OK) break;
        rc = reduce(s, true);
        if (rc != FL_OK) break;
        res = 0.0;
        for (int c = 0; c < s->nc; ++c) {
            const double r = s->h_red[s->nc + c] / ((double)m * s->h_red[2 * s->nc + c]);
            if (!(r <= res)) res = r;   // NaN propagates
        }
        if (!std::isfinite(res)) { rc = fail(s, FL_ENUMERIC, "non-finite residual"); break; }
        if (m == check_every && res < tol) break;
    }
    if (steps_done) *steps_done = done;
    if (residual) *residual = res;
    if (rc != FL_OK) return rc;
    return (res < tol) ? FL_OK : FL_ENOTCONV;
}

int fl_state_bytes(const fl_solver* s, size_t* bytes) {
    if (!s || !bytes) return FL_EINVAL;
    *bytes = 16 + s->nc * s->Q * s->N * s->pop_elem + s->D * s->N * s->pop_elem + (s->rref ? s->nc * s->N * 4 : 0);
    return FL_OK;
}

int fl_get_state_raw(fl_solver* s, void* host_buf, size_t bytes) {
    size_t need;
    if (fl_state_bytes(s, &need) != FL_OK || !host_buf || bytes < need) return FL_EINVAL;
    char* b = (char*)host_buf;
    const int64_t hdr[2] = {(int64_t)s->steps, (int64_t)need};
    std::memcpy(b, hdr, 16);
    size_t off = 16;
    const size_t pb = s->nc * s->Q * s->N * s->pop_elem;
    HIP_TRY(s, hipMemcpyAsync(b + off, s->pop[s->cur], pb, hipMemcpyDeviceToHost, s->stream));
    off += pb;
    HIP_TRY(s, hipMemcpyAsync(b + off, s->fsum[s->fcur], s->D * s->N * s->pop_elem, hipMemcpyDeviceToHost, s->stream));
    off += s->D * s->N * s->pop_elem;
    if (s->rref) HIP_TRY(s, hipMemcpyAsync(b + off, s->rref, s->nc * s->N * 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return FL_OK;
}

int fl_set_state_raw(fl_solver* s, const void* host_buf, size_t bytes) {
    size_t need;
    if (fl_state_bytes(s, &need) != FL_OK || !host_buf || bytes < need) return FL_EINVAL;
    const char* b = (const char*)host_buf;
    int64_t hdr[2];
    std::memcpy(hdr, b, 16);
    if ((size_t)hdr[1] != need) return fail(s, FL_EINVAL, "checkpoint size does not match this solver");
    size_t off = 16;
    const size_t pb = s->nc * s->Q * s->N * s->pop_elem;
    s->cur = 0;
    s->fcur = 0;
    s->fused_launches = 0;
    HIP_TRY(s, hipMemsetAsync(s->counters, 0, (size_t)8 * s->fc.cstride * sizeof(unsigned), s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->pop[0], b + off, pb, hipMemcpyHostToDevice, s->stream));
    off += pb;
    HIP_TRY(s, hipMemcpyAsync(s->fsum[0], b + off, s->D * s->N * s->pop_elem, hipMemcpyHostToDevice, s->stream));
    off += s->D * s->N * s->pop_elem;
    if (s->rref) HIP_TRY(s, hipMemcpyAsync(s->rref, b + off, s->nc * s->N * 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->steps = hdr[0];
    s->snap_valid = false;
    return FL_OK;
}

}  // extern "C"

// ===================================================================== server
#include <chrono>
#include <mutex>

namespace {

// Device staging of fl_server_result_noalloc: the velocity and pressure of one
// finished request, (D + 1) N doubles (2 MiB: requests of up to 87 381 D2Q9 or
// 65 536 D3Q19 nodes).  Every GPU the library runs on holds its own copy until
// the process ends.  Host code never uses the array's name as an address: it
// uses the pointer hipGetSymbolAddress returns for the current device.
constexpr size_t kResultScratchDoubles = size_t(1) << 18;
static __device__ __align__(256) double scratch[kResultScratchDoubles];

// This device's address of scratch, resolved once per device (with that
// device current) and kept.
hipError_t resolve_result_scratch(double** out) {
    static std::mutex mu;
    static double* per_device[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!per_device[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        per_device[dev] = static_cast<double*>(ptr);
    }
    *out = per_device[dev];
    return hipSuccess;
}

}  // namespace


namespace {
double host_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct fl_server {
    fl_solver cfg;                       // parameters, constants and launch config only
    char* pool = nullptr;
    size_t pool_bytes = 0;
    // free pool ranges (offset, size), sorted by offset, merged on free; at most
    // one more range than requests in flight, so the capacity reserved at
    // creation (max_slots + 2) is never exceeded and retiring a request
    // allocates no host memory either
    std::vector<std::pair<size_t, size_t>> free_list;
    double* result_scratch = nullptr;    // this device's static result staging (fl_server_result_noalloc)
    std::string scratch_error;
    int max_slots = 0;
    struct Req {
        uint64_t id;
        fl::SlotDesc d;
        size_t off, bytes;
        double t_submit;                 // host clock (s) when admitted
        double t_done;                   // end of the tick that saw it finish
    };
    std::vector<Req> reqs;               // running or finished-not-collected
    fl::SlotDesc* d_descs = nullptr;
    fl::SlotDesc* h_descs = nullptr;
    // per tick: block -> (request, workgroup) table and the requests' group
    // sync blocks; capacity fixed at creation
    int2* d_table = nullptr;
    int2* h_table = nullptr;
    int table_cap = 0;
    fl::GroupSync* d_sync = nullptr;
    int xcd_ok = -1;                     // blocks run on XCD (index % 8): checked at the first tick
    uint64_t next_id = 1;
    int wall_khz = 0;
    bool own_stream = false;
    std::string last_error;
};

namespace {

int sfail(fl_server* s, int code, const std::string& msg) {
    if (s) s->last_error = msg;
    return code;
}

#define SRV_TRY(s, expr)                                                                   \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) return sfail((s), FL_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

struct ReqLayout {
    size_t pop0, pop1, rt, lnf, fsum, rref, snap, total;
};

ReqLayout req_layout(const fl_solver& c, size_t N) {
    ReqLayout L{};
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += align256(b); return o; };
    const size_t pb = (size_t)c.nc * c.Q * N * c.pop_elem;
    L.pop0 = take(pb);
    L.pop1 = take(pb);
    L.rt = take((size_t)c.nc * N * 8);
    L.lnf = take((size_t)(c.nc + 1) * N * 8);
    L.fsum = take((size_t)c.D * N * c.pop_elem);
    L.rref = take(c.prm.precision == FL_FP64 ? 0 : (size_t)c.nc * N * 4);
    L.snap = take((size_t)c.nc * N * 8);
    L.total = off;
    return L;
}

bool pool_alloc(fl_server* s, size_t bytes, size_t* off) {
    for (size_t k = 0; k < s->free_list.size(); ++k) {
        auto& f = s->free_list[k];
        if (f.second >= bytes) {
            *off = f.first;
            f.first += bytes;
            f.second -= bytes;
            if (f.second == 0) s->free_list.erase(s->free_list.begin() + k);
            return true;
        }
    }
    return false;
}

void pool_free(fl_server* s, size_t off, size_t bytes) {
    auto& fl = s->free_list;
    size_t k = 0;
    while (k < fl.size() && fl[k].first < off) ++k;
    const bool join_prev = k > 0 && fl[k - 1].first + fl[k - 1].second == off;
    const bool join_next = k < fl.size() && off + bytes == fl[k].first;
    if (join_prev && join_next) {
        fl[k - 1].second += bytes + fl[k].second;
        fl.erase(fl.begin() + k);
    } else if (join_prev) {
        fl[k - 1].second += bytes;
    } else if (join_next) {
        fl[k].first = off;
        fl[k].second += bytes;
    } else {
        fl.insert(fl.begin() + k, {off, bytes});
    }
}

fl::KParams req_kparams(const fl_server* s, int nx, int ny, int nz) {
    fl::KParams kp = s->cfg.kp;
    kp.nx = nx;
    kp.ny = ny;
    kp.nz = nz;
    kp.N = nx * ny * nz;
    return kp;
}

}  // namespace

extern "C" {

int fl_server_create(const fl_params* base, size_t pool_bytes, int max_slots, void* hip_stream, fl_server** out) {
    if (!out) return FL_EINVAL;
    *out = nullptr;
    if (!base || max_slots < 1 || max_slots > 65535 || pool_bytes < 4096) return FL_EINVAL;
    fl_params p = *base;
    p.nx = p.ny = p.nz = 1;
    const int v = fl_validate(&p);
    if (v != FL_OK) return v;
    if (p.stencil != FL_STENCIL_AXIS) return FL_EINVAL;  // the server kernel has the axis stencils
    fl_server* s = new (std::nothrow) fl_server();
    if (!s) return FL_ENOMEM;
    setup(&s->cfg, &p);
    s->max_slots = max_slots;
    s->pool_bytes = pool_bytes & ~size_t(255);
    hipError_t e = hipSuccess;
    if (hip_stream) {
        s->cfg.stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&s->cfg.stream, hipStreamNonBlocking);
        s->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&s->pool, s->pool_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_descs, sizeof(fl::SlotDesc) * max_slots);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_descs, sizeof(fl::SlotDesc) * max_slots, hipHostMallocDefault);
    s->table_cap = max_slots + 8192;
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_table, sizeof(int2) * s->table_cap);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_table, sizeof(int2) * s->table_cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_sync, sizeof(fl::GroupSync) * max_slots);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fl_server_destroy(s);
        return FL_ENOMEM;
    }
    s->free_list.reserve((size_t)max_slots + 2);
    s->free_list.push_back({0, s->pool_bytes});
    // this device's result staging of fl_server_result_noalloc, resolved once
    // per device; a failure here only disables that entry point
    if (resolve_result_scratch(&s->result_scratch) != hipSuccess) {
        s->result_scratch = nullptr;
        s->scratch_error = "static result scratch: hipGetSymbolAddress failed";
        (void)hipGetLastError();
    }
    *out = s;
    return FL_OK;
}

void fl_server_destroy(fl_server* s) {
    if (!s) return;
    if (s->cfg.stream) (void)hipStreamSynchronize(s->cfg.stream);
    if (s->pool) (void)hipFree(s->pool);
    if (s->d_descs) (void)hipFree(s->d_descs);
    if (s->h_descs) (void)hipHostFree(s->h_descs);
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->h_table) (void)hipHostFree(s->h_table);
    if (s->d_sync) (void)hipFree(s->d_sync);
    if (s->own_stream && s->cfg.stream) (void)hipStreamDestroy(s->cfg.stream);
    delete s;
}

const char* fl_server_last_error(const fl_server* s) { return s ? s->last_error.c_str() : "null server"; }

int fl_server_set_tuning(fl_server* s, const char* spec) {
    if (!s) return FL_EINVAL;
    LaunchCfg lc = s->cfg.lc;
    const LaunchCfg defaults{};
    lc.serve_block = defaults.serve_block;
    lc.serve_cap = defaults.serve_cap;
    lc.serve_group = defaults.serve_group;
    if (spec && !parse_tuning(lc, spec, true))
        return sfail(s, FL_EINVAL, std::string("unknown tuning key or value in \"") + spec + "\"");
    SRV_TRY(s, hipStreamSynchronize(s->cfg.stream));
    s->cfg.lc = lc;
    return FL_OK;
}

int fl_server_request_bytes(const fl_server* s, int nx, int ny, int nz, size_t* bytes) {
    if (!s || !bytes || nx < 1 || ny < 1 || nz < 1) return FL_EINVAL;
    if (s->cfg.D == 2 && nz != 1) return FL_EINVAL;
    *bytes = req_layout(s->cfg, (size_t)nx * ny * nz).total;
    return FL_OK;
}

int fl_server_submit(fl_server* s, int nx, int ny, int nz, const double* rho_molar, double tol, long check_every,
                     long max_steps, uint64_t* id) {
    if (!s || !rho_molar || !id || check_every < 1 || max_steps < 0 || !(tol >= 0.0)) return FL_EINVAL;
    size_t bytes;
    if (fl_server_request_bytes(s, nx, ny, nz, &bytes) != FL_OK) return FL_EINVAL;
    const size_t N = (size_t)nx * ny * nz;
    if (N >= (size_t)1 << 30) return FL_EINVAL;
    const int nc = s->cfg.nc;
    std::vector<double> node(nc);
    for (size_t n = 0; n < N; ++n) {
        for (int c = 0; c < nc; ++c) node[c] = rho_molar[(size_t)c * N + n];
        if (!host_in_domain(s->cfg.kp, nc, node.data()))
            return sfail(s, FL_EDOMAIN, "initial state outside the EOS domain at node " + std::to_string(n));
    }
    if ((int)s->reqs.size() >= s->max_slots) return sfail(s, FL_EAGAIN, "no free slot");
    size_t off;
    if (!pool_alloc(s, bytes, &off)) return sfail(s, FL_EAGAIN, "pool memory exhausted");
    const ReqLayout L = req_layout(s->cfg, N);
    const fl::KParams kp = req_kparams(s, nx, ny, nz);
    fl::LaunchCfg lc = s->cfg.lc;
    lc.stream = s->cfg.stream;
    char* b = s->pool + off;
    hipError_t e = hipMemcpyAsync(b + L.rt, rho_molar, sizeof(double) * nc * N, hipMemcpyHostToDevice, lc.stream);
    float* rref = s->cfg.prm.precision == FL_FP64 ? nullptr : (float*)(b + L.rref);
    if (e == hipSuccess) e = fl::launch_init(lc, kp, (const double*)(b + L.rt), nullptr, b + L.pop0, rref, b + L.fsum);
    if (e == hipSuccess) e = fl::launch_snapshot(lc, kp, b + L.pop0, rref, (double*)(b + L.snap));
    if (e == hipSuccess) e = hipStreamSynchronize(lc.stream);
    if (e != hipSuccess) {
        pool_free(s, off, bytes);
        return sfail(s, FL_EDEVICE, std::string("submit: ") + hipGetErrorString(e));
    }
    fl_server::Req r;
    r.id = s->next_id++;
    r.off = off;
    r.bytes = bytes;
    std::memset(&r.d, 0, sizeof(r.d));
    r.d.nx = nx;
    r.d.ny = ny;
    r.d.nz = nz;
    r.d.N = (int)N;
    r.d.off_pop[0] = (long long)(off + L.pop0);
    r.d.off_pop[1] = (long long)(off + L.pop1);
    r.d.off_rt = (long long)(off + L.rt);
    r.d.off_lnf = (long long)(off + L.lnf);
    r.d.off_fsum = (long long)(off + L.fsum);
    r.d.off_rref = (long long)(off + L.rref);
    r.d.off_snap = (long long)(off + L.snap);
    r.d.max_steps = max_steps;
    r.d.check_every = check_every;
    r.d.tol = tol;
    r.d.residual = INFINITY;
    r.d.cur = 0;
    r.d.status = fl::kSlotRunning;
    r.t_submit = host_seconds();
    r.t_done = 0.0;
    s->reqs.push_back(r);
    *id = r.id;
    return FL_OK;
}

int fl_server_tick(fl_server* s, long steps, double max_ms, int* active) {
    if (!s || steps < 0) return FL_EINVAL;
    long long budget = 0;
    if (max_ms > 0.0) {
        if (s->wall_khz == 0) {
            int dev = 0, khz = 0;
            SRV_TRY(s, hipGetDevice(&dev));
            SRV_TRY(s, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
            s->wall_khz = khz > 0 ? khz : 100000;
        }
        budget = (long long)(max_ms * s->wall_khz);
        if (budget < 1) budget = 1;
    }
    std::vector<int> run, groups;
    // Advance at most as many workgroups as the device holds at once, oldest
    // request first: a workgroup beyond that would only start when another
    // leaves at the end of its time slice, and take the rest of the slice (and
    // the workgroups of one request must all be resident: they wait for each
    // other every step).
    if (s->cfg.lc.serve_cap < 0) {
        int blocks = 0;
        SRV_TRY(s, fl::serve_resident_blocks(s->cfg.lc, &blocks));
        s->cfg.lc.serve_cap = blocks > 0 ? blocks : 0;
    }
    const int cap = s->cfg.lc.serve_cap;
    // A request of more than serve_group nodes is split over up to kMaxGroup
    // workgroups of one XCD (block b runs on XCD b % 8, verified once), so
    // that its group barriers meet in one L2.
    bool grouped = s->cfg.lc.serve_group > 0 && cap >= 8 && cap % 8 == 0;
    if (grouped && s->xcd_ok < 0) s->xcd_ok = xcd_placement_ok(s->cfg.stream);
    grouped = grouped && s->xcd_ok == 1;
    int nblocks = 0;
    if (!grouped) {
        for (int k = 0; k < (int)s->reqs.size() && (cap <= 0 || (int)run.size() < cap); ++k)
            if (s->reqs[k].d.status == fl::kSlotRunning) {
                if ((int)run.size() >= s->table_cap) break;
                s->h_table[run.size()] = make_int2((int)run.size(), 0);
                run.push_back(k);
                groups.push_back(1);
            }
        nblocks = (int)run.size();
    } else {
        const int per_xcd = cap / 8;
        int used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < (int)s->reqs.size(); ++k) {
            const fl::SlotDesc& d = s->reqs[k].d;
            if (d.status != fl::kSlotRunning) continue;
            const int G = std::max(1, std::min({d.N / s->cfg.lc.serve_group, fl::kMaxGroup, per_xcd}));
            int x = -1;
            for (int c = 0; c < 8; ++c)
                if (per_xcd - used[c] >= G && (x < 0 || used[c] < used[x])) x = c;
            if (x < 0) {
                if (G == 1) break;  // every XCD is full
                continue;           // a smaller request may still fit
            }
            const int i = (int)run.size();
            for (int j = 0; j < G; ++j) s->h_table[8 * used[x]++ + x] = make_int2(i, j);
            run.push_back(k);
            groups.push_back(G);
        }
        for (int c = 0; c < 8; ++c) nblocks = std::max(nblocks, 8 * used[c]);
        for (int c = 0; c < 8; ++c)
            for (int u = used[c]; 8 * u + c < nblocks; ++u) s->h_table[8 * u + c] = make_int2(-1, 0);
    }
    const int n = (int)run.size();
    if (n > 0 && steps > 0) {
        bool any_group = false;
        for (int i = 0; i < n; ++i) {
            s->h_descs[i] = s->reqs[run[i]].d;
            s->h_descs[i].groups = groups[i];
            any_group = any_group || groups[i] > 1;
        }
        fl::LaunchCfg lc = s->cfg.lc;
        lc.stream = s->cfg.stream;
        SRV_TRY(s, hipMemcpyAsync(s->d_descs, s->h_descs, sizeof(fl::SlotDesc) * n, hipMemcpyHostToDevice, lc.stream));
        SRV_TRY(s, hipMemcpyAsync(s->d_table, s->h_table, sizeof(int2) * nblocks, hipMemcpyHostToDevice, lc.stream));
        if (any_group) SRV_TRY(s, hipMemsetAsync(s->d_sync, 0, sizeof(fl::GroupSync) * n, lc.stream));
        SRV_TRY(s, fl::launch_serve_tick(lc, s->cfg.kp, s->pool, s->d_descs, s->d_table, nblocks, s->d_sync, steps,
                                         budget));
        SRV_TRY(s, hipMemcpyAsync(s->h_descs, s->d_descs, sizeof(fl::SlotDesc) * n, hipMemcpyDeviceToHost, lc.stream));
        SRV_TRY(s, hipStreamSynchronize(lc.stream));
        const double now = host_seconds();
        for (int i = 0; i < n; ++i) {
            s->reqs[run[i]].d = s->h_descs[i];
            if (s->h_descs[i].status != fl::kSlotRunning) s->reqs[run[i]].t_done = now;
        }
    }
    if (active) {
        int a = 0;
        for (auto& r : s->reqs) a += r.d.status == fl::kSlotRunning;
        *active = a;
    }
    return FL_OK;
}

int fl_server_poll(fl_server* s, uint64_t* ids, int cap, int* n) {
    if (!s || !n || (cap > 0 && !ids)) return FL_EINVAL;
    int k = 0;
    for (auto& r : s->reqs)
        if (r.d.status != fl::kSlotRunning && k < cap) ids[k++] = r.id;
    *n = k;
    return FL_OK;
}

}  // extern "C"

namespace {

// Fields of a finished request into host arrays (any may be NULL), with u and
// p staged in dev_up ((D + 1) * N doubles of device memory).
int server_fields(fl_server* s, const fl_server::Req& r, double* dev_up, double* rho_molar, double* u, double* p) {
    const fl::KParams kp = req_kparams(s, r.d.nx, r.d.ny, r.d.nz);
    fl::LaunchCfg lc = s->cfg.lc;
    lc.stream = s->cfg.stream;
    const size_t N = r.d.N;
    const int D = s->cfg.D;
    const float* rref = s->cfg.prm.precision == FL_FP64 ? nullptr : (const float*)(s->pool + r.d.off_rref);
    hipError_t e = fl::launch_fields(lc, kp, s->pool + r.d.off_pop[r.d.cur], rref, s->pool + r.d.off_fsum,
                                     (double*)(s->pool + r.d.off_rt), dev_up, dev_up + (size_t)D * N,
                                     (double*)(s->pool + r.d.off_lnf));
    if (e == hipSuccess && rho_molar)
        e = hipMemcpyAsync(rho_molar, s->pool + r.d.off_rt, sizeof(double) * s->cfg.nc * N, hipMemcpyDeviceToHost,
                           lc.stream);
    if (e == hipSuccess && u)
        e = hipMemcpyAsync(u, dev_up, sizeof(double) * D * N, hipMemcpyDeviceToHost, lc.stream);
    if (e == hipSuccess && p)
        e = hipMemcpyAsync(p, dev_up + (size_t)D * N, sizeof(double) * N, hipMemcpyDeviceToHost, lc.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(lc.stream);
    if (e != hipSuccess) return sfail(s, FL_EDEVICE, std::string("result: ") + hipGetErrorString(e));
    return FL_OK;
}

// Index of request id among the server's requests, or -1.
int find_request(const fl_server* s, uint64_t id) {
    for (int i = 0; i < (int)s->reqs.size(); ++i)
        if (s->reqs[i].id == id) return i;
    return -1;
}

// Scalar outputs of a finished request, then its slot and memory freed.
void retire_request(fl_server* s, int k, long* steps, double* residual, int* status, double* latency_s) {
    const fl_server::Req r = s->reqs[k];
    if (steps) *steps = (long)r.d.steps;
    if (residual) *residual = r.d.residual;
    if (status)
        *status = r.d.status == fl::kSlotConverged ? FL_OK : r.d.status == fl::kSlotMaxSteps ? FL_ENOTCONV : FL_ENUMERIC;
    if (latency_s) *latency_s = r.t_done - r.t_submit;
    pool_free(s, r.off, r.bytes);
    s->reqs.erase(s->reqs.begin() + k);
}

}  // namespace

extern "C" {

int fl_server_result(fl_server* s, uint64_t id, double* rho_molar, double* u, double* p, long* steps,
                     double* residual, int* status, double* latency_s) {
    if (!s) return FL_EINVAL;
    const int k = find_request(s, id);
    if (k < 0) return sfail(s, FL_EINVAL, "unknown request id");
    const fl_server::Req& r = s->reqs[k];
    if (r.d.status == fl::kSlotRunning) return FL_EAGAIN;
    if (rho_molar || u || p) {
        double* tmp = nullptr;
        SRV_TRY(s, hipMallocAsync((void**)&tmp, sizeof(double) * (s->cfg.D + 1) * (size_t)r.d.N, s->cfg.stream));
        const int rc = server_fields(s, r, tmp, rho_molar, u, p);
        (void)hipFreeAsync(tmp, s->cfg.stream);
        if (rc != FL_OK) return rc;
    }
    retire_request(s, k, steps, residual, status, latency_s);
    return FL_OK;
}

int fl_server_result_noalloc(fl_server* s, uint64_t id, double* rho_molar, double* u, double* p, long* steps,
                             double* residual, int* status, double* latency_s) {
    if (!s) return FL_EINVAL;
    const int k = find_request(s, id);
    if (k < 0) return sfail(s, FL_EINVAL, "unknown request id");
    const fl_server::Req& r = s->reqs[k];
    if (r.d.status == fl::kSlotRunning) return FL_EAGAIN;
    if (rho_molar || u || p) {
        const size_t need = (size_t)(s->cfg.D + 1) * (size_t)r.d.N;
        if (need > kResultScratchDoubles)
            return sfail(s, FL_EINVAL, "request of " + std::to_string(r.d.N) + " nodes needs " + std::to_string(need) +
                                           " doubles of result staging, more than the static " +
                                           std::to_string(kResultScratchDoubles) + ": use fl_server_result");
        if (!s->result_scratch) return sfail(s, FL_EDEVICE, s->scratch_error);
        const int rc = server_fields(s, r, s->result_scratch, rho_molar, u, p);
        if (rc != FL_OK) return rc;
    }
    retire_request(s, k, steps, residual, status, latency_s);
    return FL_OK;
}

int fl_server_info(const fl_server* s, int* active, int* free_slots, size_t* pool_used, size_t* pool_total) {
    if (!s) return FL_EINVAL;
    int a = 0;
    size_t used = 0;
    for (auto& r : s->reqs) {
        a += r.d.status == fl::kSlotRunning;
        used += r.bytes;
    }
    if (active) *active = a;
    if (free_slots) *free_slots = s->max_slots - (int)s->reqs.size();
    if (pool_used) *pool_used = used;
    if (pool_total) *pool_total = s->pool_bytes;
    return FL_OK;
}

}  // extern "C"
