// HIP kernels of the per-step update and its auxiliary passes (gfx950).
//
// Layout in HBM (structure of arrays, node index n = x + nx*(y + ny*z)):
//   populations  g[a][n][c] for N_c <= 2: direction-major, the components of
//                             one direction of one node side by side (one
//                             vector load and one vector push store per
//                             direction and node);
//                g[c][a][n] for N_c >= 3: component-major (each component
//                             stored right after its collision: register
//                             pressure), see pop_base / pop_off;
//                             P = double, or float in the FP32 form where the
//                             rest slot a = 0 holds g_0 minus rref[n][c]
//   rt[c][n], lnf[c][n]       molar densities and ln f of the current step (FP64);
//                             plane c = N_c of lnf holds phi[n] = sum_j sqrt(kappa_j) rho~_j
//   fsum[n][k]                sum_i F_i of the previous step (population precision;
//                             read from one buffer, written to another)
//   rref[n][c]                rest-population reference (FP32 form only)
//
// Step = k_moments_eos (steps 1-5: reads every population once, writes rt and
// ln f) followed by k_collide_stream (steps 6-9: reads the node's populations,
// the rt stencil of Manhattan radius 2 and the ln f stencil of radius 1, and
// pushes the collided populations to x + e_a of the other buffer).
#include "device.h"
#include "launch.h"

namespace fl {

// Element at a 32-bit byte offset from a wave-uniform array base (every
// per-array byte offset is below 2^32: nodes < 2^29).
template <typename T>
__device__ __forceinline__ T ld(const T* base, unsigned byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st(T* base, unsigned byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Population (c, a) of node n sits at pop_base(g, c, a) + pop_off(n): a
// wave-uniform base and a 32-bit per-node byte offset.
template <int NC>
constexpr bool kInterleaved = NC <= 2;
template <int NC, int Q, typename P>
__device__ __forceinline__ const P* pop_base(const P* g, int c, int a, size_t N) {
    return kInterleaved<NC> ? g + (size_t)a * N * NC + c : g + (size_t)(c * Q + a) * N;
}
template <int NC, int Q, typename P>
__device__ __forceinline__ P* pop_base(P* g, int c, int a, size_t N) {
    return kInterleaved<NC> ? g + (size_t)a * N * NC + c : g + (size_t)(c * Q + a) * N;
}
template <int NC, typename P>
__device__ __forceinline__ unsigned pop_off(int n) {
    return (unsigned)n * (unsigned)((kInterleaved<NC> ? NC : 1) * sizeof(P));
}
template <int NC, int Q>
__device__ __forceinline__ size_t pop_index(int c, int a, size_t n, size_t N) {
    return kInterleaved<NC> ? ((size_t)a * N + n) * NC + c : ((size_t)c * Q + a) * N + n;
}

// The populations of node n; with NT through non-temporal loads (lines read
// once per pass, kept from displacing data that is read again).
template <typename L, int NC, typename P, bool NT = false>
__device__ __forceinline__ void load_pops(const P* __restrict__ g, int n, size_t N, P (&gv)[NC][L::Q]) {
    const unsigned off = pop_off<NC, P>(n);
#pragma unroll
    for (int a = 0; a < L::Q; ++a)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const P* src = reinterpret_cast<const P*>(
                reinterpret_cast<const char*>(pop_base<NC, L::Q>(g, c, a, N)) + off);
            gv[c][a] = NT ? __builtin_nontemporal_load(src) : *src;
        }
}

// rho_i = sum_a g_ai (step 1), accumulated in FP64; also sum of the moving ones.
// ref[c] is the node's rest-population reference (FP32 form; unused in FP64).
template <typename L, typename P>
__device__ __forceinline__ void comp_density(const P (&gv)[L::Q], float ref, double& rho, double& moving) {
    double m = 0.0;
#pragma unroll
    for (int a = 1; a < L::Q; ++a) m += (double)gv[a];
    double r0 = (double)gv[0];
    if constexpr (sizeof(P) == 4) r0 += (double)ref;
    moving = m;
    rho = r0 + m;
}

template <typename L, int NC, typename P>
__device__ __forceinline__ void densities_ref(const P (&gv)[NC][L::Q], const float (&ref)[NC], double (&rho)[NC],
                                              double (&moving)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) comp_density<L, P>(gv[c], ref[c], rho[c], moving[c]);
}

// Momentum sum_a e_a g_a of one component in FP64 (step 1).
template <typename L, typename P>
__device__ __forceinline__ void comp_momentum(const P (&gv)[L::Q], double (&j)[3]) {
    j[0] = j[1] = j[2] = 0.0;
    Unroll<0, L::Q>::run([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        if constexpr (L::ex[a] != 0) j[0] += (double)gv[a] * L::ex[a];
        if constexpr (L::ey[a] != 0) j[1] += (double)gv[a] * L::ey[a];
        if constexpr (L::ez[a] != 0) j[2] += (double)gv[a] * L::ez[a];
    });
}

template <int NC, typename P>
__device__ __forceinline__ void load_ref(const float* __restrict__ rref, int n, float (&ref)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) ref[c] = sizeof(P) == 4 ? ld(rref, ((unsigned)n * NC + c) * 4u) : 0.f;
}

template <typename L, int NC, typename P>
__device__ __forceinline__ void densities(const P (&gv)[NC][L::Q], const float* __restrict__ rref, int n,
                                          size_t N, double (&rho)[NC], double (&moving)[NC]) {
    float ref[NC];
    load_ref<NC, P>(rref, n, ref);
    densities_ref<L, NC, P>(gv, ref, rho, moving);
}

// Node of this thread, or -1.  With xcd_chunk > 0 the hardware block b
// (dispatched round-robin over the 8 XCDs) handles logical block
// (b % 8) * xcd_chunk + b / 8, so every XCD sweeps one contiguous range of nodes
// and its L2 keeps the neighbouring planes the stencil needs.  With rev the
// logical blocks run from the last node to the first: a pass that follows one
// sweeping the other way starts on the lines that pass touched last, which the
// memory-side cache still holds.
__device__ __forceinline__ int node_index(int xcd_chunk, int N, bool rev = false) {
    const int b = blockIdx.x;
    int lb = xcd_chunk > 0 ? (b & 7) * xcd_chunk + (b >> 3) : b;
    if (rev) lb = (N + (int)blockDim.x - 1) / (int)blockDim.x - 1 - lb;
    const int n = lb * (int)blockDim.x + (int)threadIdx.x;
    return (lb < 0 || n >= N) ? -1 : n;
}

// Visiting order of the nodes: the k-th node visited is slab_order(k).  The
// x-lines (rows) of the lattice are taken slab by slab, zs planes per slab,
// and y-major inside a slab (z fastest), so the planes z +- 2 a node's stencil
// reaches are visited together and the rows y +- 2 shortly before: the FP64
// fields they hold are re-read from L2 instead of memory.  A bijection of
// [0, N) for any nz, zs >= 1; zs <= 0 keeps the plain order.
__device__ __forceinline__ int slab_order(int k, int nx, int ny, int nz, int zs) {
    if (zs <= 0 || k < 0) return k;
    const int x = k % nx;
    const int r = k / nx;               // row in visiting order
    const int per = ny * zs;            // rows per slab
    const int sl = r / per;
    const int p = r - sl * per;
    const int zlen = min(zs, nz - sl * zs);
    const int y = p / zlen;
    const int z = sl * zs + (p - y * zlen);
    return x + nx * (y + ny * z);
}

// XCD-band visiting order: hardware block b runs on XCD b % 8.  The rows of
// every plane are cut into `bands` bands (a multiple of 8); XCD k sweeps its
// bands k, k + 8, ... one after the other, each one plane at a time along z
// (rows, then x, inside a band-plane; planes downward with rev).  The planes
// z - 1, z, z + 1 a node's stencil reaches are then the band's last three,
// whose FP64 fields fit in the XCD's L2, instead of the last three whole
// planes, which do not.  A bijection of [0, N) for any extents (a band may be
// empty when ny < bands); -1 for a thread past its band.
__device__ __forceinline__ int band_node(int nx, int ny, int nz, int bands, bool rev) {
    const int b = blockIdx.x;
    const int k = b & 7, j = b >> 3;
    const int bs = (int)blockDim.x;
    const int maxrows = (ny + bands - 1) / bands;
    const int bpp = (maxrows * nx + bs - 1) / bs;   // blocks per band-plane
    const int m = j / (bpp * nz);                   // which of the XCD's bands
    if (m >= (bands >> 3)) return -1;
    const int r = j - m * bpp * nz;
    int z = r / bpp;
    const int q = k + 8 * m;
    const int Y0 = (int)((long long)q * ny / bands), Y1 = (int)((long long)(q + 1) * ny / bands);
    const int pos = (r - z * bpp) * bs + (int)threadIdx.x;
    if (pos >= (Y1 - Y0) * nx) return -1;
    if (rev) z = nz - 1 - z;
    return pos % nx + nx * (Y0 + pos / nx + ny * z);
}

// Blocks of a band-ordered launch (see band_node).
static inline int band_grid(int nx, int ny, int nz, int bands, int bs) {
    const int maxrows = (ny + bands - 1) / bands;
    return bands * ((maxrows * nx + bs - 1) / bs) * nz;
}

// Lattice extent (per solver, or per request in the batched server).
struct Dims {
    int nx, ny, nz, N;
};

// ----------------------------------------------------------------- step 1-5
// Steps 1-5 at node n: densities, molar densities, mixing, EOS, ln f.
template <int LAT, int NC, typename P, bool NTLD = false>
__device__ __forceinline__ bool node_moments_eos(const KParams& kp, int n, size_t N, const P* __restrict__ g,
                                                 const float* __restrict__ rref, double* __restrict__ rt,
                                                 double* __restrict__ lnf) {
    using L = Lat<LAT>;
    P gv[NC][L::Q];
    load_pops<L, NC, P, NTLD>(g, n, N, gv);
    double rho[NC], mov[NC], r[NC], lf[NC];
    densities<L, NC, P>(gv, rref, n, N, rho, mov);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        r[c] = rho[c] / kp.M[c];
        rt[(size_t)c * N + n] = r[c];
    }
    const bool ok = eos_lnf<NC>(kp, r, lf, nullptr);
    double phi = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        lnf[(size_t)c * N + n] = lf[c];
        phi += kp.sk[c] * r[c];
    }
    lnf[(size_t)NC * N + n] = phi;
    return ok;
}

template <int LAT, int NC, typename P>
__global__ __launch_bounds__(256) void k_moments_eos(KParams kp, const P* __restrict__ g,
                                                     const float* __restrict__ rref,
                                                     double* __restrict__ rt, double* __restrict__ lnf,
                                                     int* __restrict__ err, int xcd_chunk, int zs) {
    const int n = slab_order(node_index(xcd_chunk, kp.N), kp.nx, kp.ny, kp.nz, zs);
    if (n < 0) return;
    // non-temporal population loads: each line is read once by this pass (faster
    // by about a sixth on the 128^3 binary lattice; the collide pass after it is
    // not slowed)
    if (!node_moments_eos<LAT, NC, P, true>(kp, n, kp.N, g, rref, rt, lnf)) atomicOr(err, 1);
}

// Steps 1-5 at two consecutive nodes n0, n0 + 1 per thread (N_c >= 3, FP32
// populations in the component-major layout, N even): each population stream
// is read 8 bytes per lane, so a wave's load covers four whole 128-byte lines
// instead of two; the per-node arithmetic is that of node_moments_eos, so the
// fields are the same bit for bit.
typedef float fl_f2 __attribute__((ext_vector_type(2)));
typedef double fl_d2 __attribute__((ext_vector_type(2)));

template <int LAT, int NC>
__device__ __forceinline__ bool node_fields(const KParams& kp, const float (&gv)[NC][Lat<LAT>::Q],
                                            const float* __restrict__ rref, int n, size_t N, double (&r)[NC],
                                            double (&lf)[NC], double& phi) {
    using L = Lat<LAT>;
    double rho[NC], mov[NC];
    densities<L, NC, float>(gv, rref, n, N, rho, mov);
#pragma unroll
    for (int c = 0; c < NC; ++c) r[c] = rho[c] / kp.M[c];
    const bool ok = eos_lnf<NC>(kp, r, lf, nullptr);
    phi = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) phi += kp.sk[c] * r[c];
    return ok;
}

template <int LAT, int NC>
__global__ __launch_bounds__(256) void k_moments_eos_pair(KParams kp, const float* __restrict__ g,
                                                          const float* __restrict__ rref,
                                                          double* __restrict__ rt, double* __restrict__ lnf,
                                                          int* __restrict__ err) {
    static_assert(!kInterleaved<NC>, "component-major layout only");
    using L = Lat<LAT>;
    const int n0 = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (n0 >= kp.N) return;  // N even: n0 + 1 < N as well
    const size_t N = kp.N;
    float gv0[NC][L::Q], gv1[NC][L::Q];
#pragma unroll
    for (int a = 0; a < L::Q; ++a)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // non-temporal: each line is read once by this pass
            const fl_f2 v = __builtin_nontemporal_load(
                reinterpret_cast<const fl_f2*>(pop_base<NC, L::Q>(g, c, a, N) + n0));
            gv0[c][a] = v.x;
            gv1[c][a] = v.y;
        }
    double r0[NC], r1[NC], lf0[NC], lf1[NC], phi0, phi1;
    const bool ok0 = node_fields<LAT, NC>(kp, gv0, rref, n0, N, r0, lf0, phi0);
    const bool ok1 = node_fields<LAT, NC>(kp, gv1, rref, n0 + 1, N, r1, lf1, phi1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        *reinterpret_cast<fl_d2*>(rt + (size_t)c * N + n0) = fl_d2{r0[c], r1[c]};
        *reinterpret_cast<fl_d2*>(lnf + (size_t)c * N + n0) = fl_d2{lf0[c], lf1[c]};
    }
    *reinterpret_cast<fl_d2*>(lnf + (size_t)NC * N + n0) = fl_d2{phi0, phi1};
    if (!(ok0 && ok1)) atomicOr(err, 1);
}

// ---------------------------------------------------------------- step 6-9
// wrap v into [0, m) for |v - [0, m)| <= 2m (stencil offsets of at most 2)
__device__ __forceinline__ int wrap2(int v, int m) {
    v = v < 0 ? v + m : v;
    v = v < 0 ? v + m : v;
    v = v >= m ? v - m : v;
    return v >= m ? v - m : v;
}

__device__ __forceinline__ void unit_offset(int k, int s, int& dx, int& dy, int& dz) {
    dx = (k == 0) ? s : 0;
    dy = (k == 1) ? s : 0;
    dz = (k == 2) ? s : 0;
}

// Steps 6-7 at one node from accessors of the FP64 fields of the moments pass:
// phi_at(dx,dy,dz) (Manhattan radius 2), rt_at(i,dx,dy,dz) and
// lnf_at(i,dx,dy,dz) (radius 1).  Every offset is a compile-time constant after
// unrolling, so an accessor resolves to one global, LDS or register read.
//   step 6: with kappa_ij = sqrt(kappa_i kappa_j) (eqkappa),
//     mu_I,i = -sum_j kappa_ij lap(rho~_j) = -sqrt(kappa_i) lap(phi),
//     phi = sum_j sqrt(kappa_j) rho~_j: one scalar Laplacian (eq2ndder per
//     axis) at each of the 2D neighbours;
//   step 7: F_i = -rho~_i [RT D(ln f_i) + D(mu_I,i)] and grad rho_i by central
//     differences (eq1stder).
// F and G are evaluated in FP64 and kept in the collision precision T (the
// collision reads them there); their sum over components stays FP64.
template <int D, int NC, typename T, class PhiAt, class RtAt, class LnfAt>
__device__ __forceinline__ void stencil_force(const KParams& kp, PhiAt&& phi_at, RtAt&& rt_at, LnfAt&& lnf_at,
                                              T (&F)[NC][3], T (&G)[NC][3], double (&Fs)[3]) {
    double mh[2 * D];  // -lap(phi) at n + e_k (index 2k) and n - e_k (index 2k+1)
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            int cx, cy, cz;
            unit_offset(k, s == 0 ? 1 : -1, cx, cy, cz);
            const double p0 = phi_at(cx, cy, cz);
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < D; ++m) {
                int mx, my, mz;
                unit_offset(m, 1, mx, my, mz);
                acc += phi_at(cx + mx, cy + my, cz + mz) - 2.0 * p0 + phi_at(cx - mx, cy - my, cz - mz);
            }
            mh[2 * k + s] = -acc;
        }
#pragma unroll
    for (int k = 0; k < 3; ++k) Fs[k] = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const double rc = rt_at(i, 0, 0, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            F[i][k] = T(0);
            G[i][k] = T(0);
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            int px, py, pz;
            unit_offset(k, 1, px, py, pz);
            const double dl = (lnf_at(i, px, py, pz) - lnf_at(i, -px, -py, -pz)) / 2.0;
            const double dm = kp.sk[i] * (mh[2 * k] - mh[2 * k + 1]) / 2.0;
            double f = -rc * (kp.RT * dl + dm);
            const double gr = kp.M[i] * (rt_at(i, px, py, pz) - rt_at(i, -px, -py, -pz)) / 2.0;
            if constexpr (sizeof(T) == 8)
                if (kp.standard) f += gr / 3.0;  // eqForceGen: + c_s^2 grad rho_i
            Fs[k] += f;
            F[i][k] = T(f);
            G[i][k] = T(gr);
        }
    }
}

// Steps 6-7 with the isotropic lattice stencils, an option beside the axis
// differences of eq1stder and eq2ndder (with those, a 3-D sphere leaves the EOS
// domain; with these it relaxes): with the lattice weights w_a and c_s^2 = 1/3,
//   grad f(n) = (1/c_s^2) sum_a w_a e_a f(n + e_a),
//   lap f(n)  = (2/c_s^2) sum_a w_a (f(n + e_a) - f(n)).
// On a field that varies along one axis only they are the axis differences.
//
// -lap(phi) of the isotropic stencil at one point from an accessor
// phi_at(dx, dy, dz); shared by the Laplacian pass (global memory) and the
// z-marching collide kernel (LDS), so both give the same bits.
template <int LAT, class PhiAt>
__device__ __forceinline__ double neg_lap_iso(PhiAt&& phi_at) {
    using L = Lat<LAT>;
    constexpr double cs2 = 1.0 / 3.0;
    const double p0 = phi_at(0, 0, 0);
    double acc = 0.0;
#pragma unroll
    for (int b = 1; b < L::Q; ++b) acc = __builtin_fma(L::w[b], phi_at(L::ex[b], L::ey[b], L::ez[b]) - p0, acc);
    return -(2.0 * acc / cs2);
}

// mu_i = RT ln f_i + mu_I,i at one point, mu_I,i = sqrt(kappa_i) (-lap(phi))
// (steps 5-6): F_i = -rho~_i grad(mu_i) is the force of eqforceFugLBM.
__device__ __forceinline__ double chem_pot(const KParams& kp, int i, double lnf, double mh) {
    return __builtin_fma(kp.RT, lnf, kp.sk[i] * mh);
}

// The D3Q19 isotropic gradient split by planes.  With the weights 1/18 (axis)
// and 1/36 (edges), grad f(x, y, z) = (1/12) (
//   x: 2 Ax(z) + Ax(y+1, z) + Ax(y-1, z) + Ax(z+1) + Ax(z-1),
//   y: 2 Ay(z) + Ay(x+1, z) + Ay(x-1, z) + Ay(z+1) + Ay(z-1),
//   z: B(z+1) - B(z-1) ),
// Ax = f(x+1) - f(x-1) and Ay = f(y+1) - f(y-1) in one plane, and B = 2 f +
// (f(x+1) + f(x-1)) + (f(y+1) + f(y-1)) in one plane.  A node's own plane
// gives Sx = 2 Ax + (Ax(y+1) + Ax(y-1)) and Sy (its 3 x 3 points); each of the
// planes z +- 1 gives Ax, Ay and B at the node's column (its cross).  The
// z-marching kernel computes these from each plane as it passes and keeps
// them per node, the one-thread-per-node kernel from its neighbours: the same
// expressions, combined in the same order, give the same bits.
struct IsoCross {
    double ax, ay, b;
};
struct IsoOwn {
    double sx, sy, c;
};

template <class At>
__device__ __forceinline__ IsoCross iso_cross(At&& f) {
    IsoCross r;
    r.ax = f(1, 0) - f(-1, 0);
    r.ay = f(0, 1) - f(0, -1);
    const double c = f(0, 0);
    r.b = (c + c) + ((f(1, 0) + f(-1, 0)) + (f(0, 1) + f(0, -1)));
    return r;
}

template <class At>
__device__ __forceinline__ IsoOwn iso_own(At&& f) {
    IsoOwn r;
    const double ax = f(1, 0) - f(-1, 0);
    const double ay = f(0, 1) - f(0, -1);
    r.sx = (ax + ax) + ((f(1, 1) - f(-1, 1)) + (f(1, -1) - f(-1, -1)));
    r.sy = (ay + ay) + ((f(1, 1) - f(1, -1)) + (f(-1, 1) - f(-1, -1)));
    r.c = f(0, 0);
    return r;
}

// Gradient at z from the partial sums Sx(z) + Ax(z-1), Sy(z) + Ay(z-1), the
// plane below's B and the plane above's cross (times 1/12 rounded, not a
// division: a multiply instead of a division sequence in FP64).
__device__ __forceinline__ void iso_grad(double px, double py, double bm, const IsoCross& up, double (&g)[3]) {
    constexpr double kTwelfth = 1.0 / 12.0;
    g[0] = (px + up.ax) * kTwelfth;
    g[1] = (py + up.ay) * kTwelfth;
    g[2] = (up.b - bm) * kTwelfth;
}

// F_i = -rho~_i grad(mu_i), grad rho_i = M_i grad(rho~_i) (step 7), from the
// gradients of mu_i and rho~_i and the node's rho~_i, kept in the collision
// precision T; their sum over components in FP64.
// One component i: f = F_i in FP64 (summed over components by the caller), F_i
// and grad rho_i in T.
template <typename T>
__device__ __forceinline__ void comp_force(const KParams& kp, int i, const double (&gmu)[3], const double (&grt)[3],
                                           double rc, double (&f)[3], T (&F)[3], T (&G)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double fk = -(rc * gmu[k]);
        const double gr = kp.M[i] * grt[k];
        if constexpr (sizeof(T) == 8)
            if (kp.standard) fk += gr / 3.0;  // eqForceGen: + c_s^2 grad rho_i
        f[k] = fk;
        F[k] = T(fk);
        G[k] = T(gr);
    }
}

template <int NC, typename T>
__device__ __forceinline__ void force_from_grads(const KParams& kp, const double (&gmu)[NC][3],
                                                 const double (&grt)[NC][3], const double (&rc)[NC],
                                                 T (&F)[NC][3], T (&G)[NC][3], double (&Fs)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) Fs[k] = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        double f[3];
        comp_force<T>(kp, i, gmu[i], grt[i], rc[i], f, F[i], G[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) Fs[k] += f[k];
    }
}

// Steps 6-7 at one node of a D3Q19 lattice with the isotropic stencils, from
// accessors mu_at(i, dx, dy, dz) of mu_i and rt_at(i, dx, dy, dz) of rho~_i at
// the node's D3Q19 neighbours: the gradients by planes (iso_own at the node's
// plane, iso_cross at the planes below and above), then the forces.
// With SERIAL, the instruction scheduler may not move work across components
// (it would otherwise issue every component's stencil reads at once, which
// costs registers); the arithmetic is the same either way.
template <int NC, typename T, bool SERIAL = false, class MuAt, class RtAt>
__device__ __forceinline__ void stencil_force_iso_mu(const KParams& kp, MuAt&& mu_at, RtAt&& rt_at, T (&F)[NC][3],
                                                     T (&G)[NC][3], double (&Fs)[3]) {
    double gmu[NC][3], grt[NC][3], rc[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        if constexpr (SERIAL) __builtin_amdgcn_sched_barrier(0);
        auto mu = [&](int dz) { return [&, dz](int dx, int dy) { return mu_at(i, dx, dy, dz); }; };
        auto r = [&](int dz) { return [&, dz](int dx, int dy) { return rt_at(i, dx, dy, dz); }; };
        const IsoCross mdn = iso_cross(mu(-1)), mup = iso_cross(mu(1));
        const IsoOwn mown = iso_own(mu(0));
        iso_grad(mown.sx + mdn.ax, mown.sy + mdn.ay, mdn.b, mup, gmu[i]);
        const IsoCross rdn = iso_cross(r(-1)), rup = iso_cross(r(1));
        const IsoOwn rown = iso_own(r(0));
        iso_grad(rown.sx + rdn.ax, rown.sy + rdn.ay, rdn.b, rup, grt[i]);
        rc[i] = rown.c;
    }
    force_from_grads<NC, T>(kp, gmu, grt, rc, F, G, Fs);
}

// Steps 6-7 at one node with the isotropic stencils, from accessors of the
// fields of the moments pass: mh_at(dx,dy,dz) = -lap(phi) (from the Laplacian
// pass), rt_at and lnf_at as for stencil_force.
template <int LAT, int NC, typename T, class MhAt, class RtAt, class LnfAt>
__device__ __forceinline__ void stencil_force_iso(const KParams& kp, MhAt&& mh_at, RtAt&& rt_at, LnfAt&& lnf_at,
                                                  T (&F)[NC][3], T (&G)[NC][3], double (&Fs)[3]) {
    using L = Lat<LAT>;
    constexpr int D = L::D, Q = L::Q;
    if constexpr (D == 3) {
        stencil_force_iso_mu<NC, T>(
            kp, [&](int i, int dx, int dy, int dz) { return chem_pot(kp, i, lnf_at(i, dx, dy, dz), mh_at(dx, dy, dz)); },
            rt_at, F, G, Fs);
    } else {
        constexpr double cs2 = 1.0 / 3.0;
        double mh[Q];  // -lap(phi) at n + e_a
        mh[0] = 0.0;
#pragma unroll
        for (int a = 1; a < Q; ++a) mh[a] = mh_at(L::ex[a], L::ey[a], L::ez[a]);
#pragma unroll
        for (int k = 0; k < 3; ++k) Fs[k] = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double rc = rt_at(i, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                F[i][k] = T(0);
                G[i][k] = T(0);
            }
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double sl = 0.0, sm = 0.0, sg = 0.0;
#pragma unroll
                for (int a = 1; a < Q; ++a) {
                    const int e = k == 0 ? L::ex[a] : (k == 1 ? L::ey[a] : L::ez[a]);
                    if (e == 0) continue;
                    const double we = L::w[a] * e;
                    sl += we * lnf_at(i, L::ex[a], L::ey[a], L::ez[a]);
                    sm += we * mh[a];
                    sg += we * rt_at(i, L::ex[a], L::ey[a], L::ez[a]);
                }
                const double dl = sl / cs2;
                const double dm = kp.sk[i] * (sm / cs2);
                double f = -rc * (kp.RT * dl + dm);
                const double gr = kp.M[i] * (sg / cs2);
                if constexpr (sizeof(T) == 8)
                    if (kp.standard) f += gr / 3.0;  // eqForceGen: + c_s^2 grad rho_i
                Fs[k] += f;
                F[i][k] = T(f);
                G[i][k] = T(gr);
            }
        }
    }
}

// The node's own inputs of steps 8-9: its populations, its rest-population
// reference (FP32 form) and the previous step's force sum.  With NTLD the
// populations are loaded with the non-temporal hint: each is read once per
// pass, and keeping them out of the way leaves L2 to the FP64 stencil fields
// that neighbouring nodes re-read.
template <int LAT, int NC, typename P>
struct NodeIn {
    P gv[NC][Lat<LAT>::Q];
    P fprev[3];
    float ref[NC];
};

template <int LAT, int NC, typename P, bool NTLD>
__device__ __forceinline__ void load_node_inputs(const P* __restrict__ g, const P* fsum_in,
                                                 const float* __restrict__ rref, int n, size_t N,
                                                 NodeIn<LAT, NC, P>& in) {
    using L = Lat<LAT>;
    constexpr int D = L::D, Q = L::Q;
#pragma unroll
    for (int k = 0; k < D; ++k) in.fprev[k] = ld(fsum_in, ((unsigned)n * D + k) * (unsigned)sizeof(P));
    load_pops<L, NC, P, NTLD>(g, n, N, in.gv);
    load_ref<NC, P>(rref, n, in.ref);
}

// Periodic neighbour n + e of node n = (x, y, z) as n plus per-axis steps
// (wrapped at the faces); off() gives the byte offset of its populations.
template <int D, int NC, typename P>
struct PushGeom {
    int n;
    int step[3][2];
    __device__ __forceinline__ PushGeom(const Dims& dm, int n_, int x, int y, int z) : n(n_) {
        const int nx = dm.nx, sy = dm.nx, sz = dm.nx * dm.ny;
        step[0][0] = x == 0 ? nx - 1 : -1;
        step[0][1] = x == nx - 1 ? 1 - nx : 1;
        step[1][0] = y == 0 ? (dm.ny - 1) * sy : -sy;
        step[1][1] = y == dm.ny - 1 ? (1 - dm.ny) * sy : sy;
        step[2][0] = z == 0 ? (dm.nz - 1) * sz : -sz;
        step[2][1] = z == dm.nz - 1 ? (1 - dm.nz) * sz : sz;
    }
    __device__ __forceinline__ unsigned off(int dx, int dy, int dz) const {
        int m = n;
        if (dx) m += step[0][dx > 0];
        if (dy) m += step[1][dy > 0];
        if (D == 3 && dz) m += step[2][dz > 0];
        return pop_off<NC, P>(m);
    }
};

// Step 1's velocity from the node's densities rho_i and momentum j (FP64) and
// the force of the chosen time level: this step's sum Fs or the previous
// step's fprev.
template <int D, typename P>
__device__ __forceinline__ void node_velocity(const KParams& kp, double rtot, const double (&j)[3],
                                              const double (&Fs)[3], const P (&fprev)[3], double (&u)[3]) {
    u[0] = u[1] = u[2] = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double fk = kp.force_level ? Fs[k] : (double)fprev[k];
        u[k] = (j[k] + 0.5 * fk) / rtot;
    }
}

// Which form of the collision a lattice of N_c components in precision P
// runs (every kernel of one N_c and precision the same, so they agree bit for
// bit): the pair form (collide_pairs) with FP64 populations, where the
// three-component isotropic z-march measured 4.33 -> 3.94 ms with it on the
// 256^3 ternary lattice; the direction-by-direction one (collide) with FP32
// populations, where the pair form made the three-component split pass
// slower (2.31 -> 2.43 ms, same box) and left the 128^3 binary z-march and the
// batched server as they were.
template <int NC, typename P>
constexpr bool kPairCollision = sizeof(P) == 8;

// Steps 8-9 of component c at a node: equilibrium, forcing and collision of
// its populations gv (stored convention, see collide), result in oc.
template <typename L, typename P, bool MRT, bool PAIRS>
__device__ __forceinline__ void collide_comp(const KParams& kp, const P (&gv)[L::Q], double rho, double mov,
                                             const double (&u)[3], const P (&F)[3], const P (&G)[3],
                                             P (&oc)[L::Q]) {
    using T = P;  // collision precision
    CompState<T> cs;
    cs.rho = T(rho);
    cs.ux = T(u[0]); cs.uy = T(u[1]); cs.uz = T(u[2]);
    cs.Fx = F[0]; cs.Fy = F[1]; cs.Fz = F[2];
    cs.Gx = G[0]; cs.Gy = G[1]; cs.Gz = G[2];
    bool std_form = false;
    if constexpr (sizeof(P) == 8) std_form = kp.standard != 0;
    if constexpr (sizeof(P) == 8) {
        if (std_form) {
            cs.Gx = cs.Gy = cs.Gz = T(0);  // Guo forcing without the grad rho part
            if constexpr (PAIRS)
                collide_pairs<L, T, MRT, false, true>(kp, cs, gv, T(mov), oc);
            else
                collide<L, T, MRT, false, true>(kp, cs, gv, T(mov), oc);
        }
    }
    if (!std_form) {
        if constexpr (PAIRS)
            collide_pairs<L, T, MRT, (sizeof(P) == 4)>(kp, cs, gv, T(mov), oc);
        else
            collide<L, T, MRT, (sizeof(P) == 4)>(kp, cs, gv, T(mov), oc);
    }
}

// Push of component c's post-collision populations to n + e_a of gn
// (component-major layout).
template <typename L, int NC, typename P>
__device__ __forceinline__ void push_comp(const PushGeom<L::D, NC, P>& pg, P* __restrict__ gn, int c, size_t N,
                                          const P (&o)[L::Q], bool nt) {
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
        P* dst = pop_base<NC, L::Q>(gn, c, a, N);
        const unsigned off = pg.off(L::ex[a], L::ey[a], L::ez[a]);
        if (nt)
            __builtin_nontemporal_store(o[a], (P*)((char*)dst + off));
        else
            st(dst, off, o[a]);
    }
}

// Steps 8-9 (and step 1's velocity) at node n = (x, y, z) from its loaded
// inputs (gv, fprev): moments of the node's populations, u with the force of
// the chosen time level, equilibrium, forcing and collision per component, push
// streaming to n + e_a of gn.  The momentum is summed component by component
// for N_c >= 3 (each component's sum first, then their sum in order), so a
// kernel that gives each component to its own threads forms the same bits.
template <int LAT, int NC, typename P, bool MRT>
__device__ __forceinline__ void collide_push_loaded(const KParams& kp, const Dims& dm, int n, int x, int y, int z,
                                                    const NodeIn<LAT, NC, P>& in, P* __restrict__ gn,
                                                    const P (&F)[NC][3], const P (&G)[NC][3],
                                                    const double (&Fs)[3], P* fsum_out, bool nt) {
    using L = Lat<LAT>;
    const auto& gv = in.gv;
    constexpr int D = L::D, Q = L::Q;
    using T = P;  // collision precision
    const size_t N = dm.N;
    const PushGeom<D, NC, P> pg(dm, n, x, y, z);

    double rho[NC], mov[NC];
    densities_ref<L, NC, P>(gv, in.ref, rho, mov);
    double rtot = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        rtot += rho[c];
        if constexpr (NC >= 3) {
            double jc[3];
            comp_momentum<L, P>(gv[c], jc);
#pragma unroll
            for (int k = 0; k < 3; ++k) j[k] += jc[k];
        } else {
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                j[0] += (double)gv[c][a] * L::ex[a];
                j[1] += (double)gv[c][a] * L::ey[a];
                j[2] += (double)gv[c][a] * L::ez[a];
            }
        }
    }
    double u[3];
    node_velocity<D, P>(kp, rtot, j, Fs, in.fprev, u);
    // Push: direction a goes to n + e_a.  With the interleaved layout (N_c <= 2)
    // both values of a direction leave as one vector store (all outputs live
    // at once); with more components each is stored right after its collision.
    constexpr bool kJoint = kInterleaved<NC>;
    T out[kJoint ? NC : 1][Q];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T (&oc)[Q] = out[kJoint ? c : 0];
        collide_comp<L, P, MRT, kPairCollision<NC, P>>(kp, gv[c], rho[c], mov[c], u, F[c], G[c], oc);
        if constexpr (!kJoint) push_comp<L, NC, P>(pg, gn, c, N, oc, nt);
    }
    if constexpr (kJoint) {
        using V = P __attribute__((ext_vector_type(NC)));
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            V v;
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = out[c][a];
            V* dst = reinterpret_cast<V*>(reinterpret_cast<char*>(pop_base<NC, Q>(gn, 0, a, N)) +
                                          pg.off(L::ex[a], L::ey[a], L::ez[a]));
            if (nt)
                __builtin_nontemporal_store(v, dst);
            else
                *dst = v;
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) st(fsum_out, ((unsigned)n * D + k) * (unsigned)sizeof(P), (P)Fs[k]);
}

// Steps 8-9 at node n, loading its inputs first.  The force sum of the previous
// step is loaded whichever time level u takes: loaded inside that choice, it
// was issued only after the populations had arrived (one more memory latency
// per node).
template <int LAT, int NC, typename P, bool MRT, bool NTLD = false>
__device__ __forceinline__ void collide_push(const KParams& kp, const Dims& dm, int n, int x, int y, int z,
                                             const P* __restrict__ g, P* __restrict__ gn,
                                             const float* __restrict__ rref, const P (&F)[NC][3],
                                             const P (&G)[NC][3], const double (&Fs)[3], const P* fsum_in,
                                             P* fsum_out, bool nt) {
    NodeIn<LAT, NC, P> in;
    load_node_inputs<LAT, NC, P, NTLD>(g, fsum_in, rref, n, dm.N, in);
    collide_push_loaded<LAT, NC, P, MRT>(kp, dm, n, x, y, z, in, gn, F, G, Fs, fsum_out, nt);
}

// Steps 6-9 at node n reading the FP64 fields straight from global memory.
template <int LAT, int NC, typename P, bool MRT, bool NTLD = false, bool ISO = false>
__device__ __forceinline__ void node_collide_stream(const KParams& kp, const Dims& dm, int n,
                                                    const P* __restrict__ g, P* __restrict__ gn,
                                                    const float* __restrict__ rref,
                                                    const double* __restrict__ rt,
                                                    const double* __restrict__ lnf,
                                                    const P* fsum_in, P* fsum_out, bool nt) {
    using L = Lat<LAT>;
    constexpr int D = L::D;
    const size_t N = dm.N;
    const int nx = dm.nx, ny = dm.ny, nz = dm.nz;
    const int x = n % nx;
    const int t = n / nx;
    const int y = t % ny;
    const int z = t / ny;
    int X[5], Y[5], Z[5];
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        X[d + 2] = wrap2(x + d, nx);
        Y[d + 2] = wrap2(y + d, ny);
        Z[d + 2] = (D == 3) ? wrap2(z + d, nz) : 0;
    }
    auto idx = [&](int dx, int dy, int dz) { return X[dx + 2] + nx * (Y[dy + 2] + ny * Z[dz + 2]); };
    const double* phi = lnf + (size_t)NC * N;
    P F[NC][3], G[NC][3];
    double Fs[3];
    auto phi_at = [&](int dx, int dy, int dz) { return phi[idx(dx, dy, dz)]; };
    auto rt_at = [&](int i, int dx, int dy, int dz) { return rt[(size_t)i * N + idx(dx, dy, dz)]; };
    auto lnf_at = [&](int i, int dx, int dy, int dz) { return lnf[(size_t)i * N + idx(dx, dy, dz)]; };
    if constexpr (ISO) {
        const double* mh = phi + N;  // -lap(phi) of k_interface_lap
        stencil_force_iso<LAT, NC, P>(
            kp, [&](int dx, int dy, int dz) { return mh[idx(dx, dy, dz)]; }, rt_at, lnf_at, F, G, Fs);
    } else {
        stencil_force<D, NC, P>(kp, phi_at, rt_at, lnf_at, F, G, Fs);
    }
    collide_push<LAT, NC, P, MRT, NTLD>(kp, dm, n, x, y, z, g, gn, rref, F, G, Fs, fsum_in, fsum_out, nt);
}

// -lap(phi) of the isotropic stencils at every node (phi = sum_j sqrt(kappa_j)
// rho~_j from the moments pass); read by the collide pass at n + e_a.
// Consecutive rows go to one XCD (xcd_chunk), so that the rows y +- 1 a row
// reads are in that XCD's L2.
template <int LAT>
__global__ __launch_bounds__(256) void k_interface_lap(const double* __restrict__ phi, double* __restrict__ mh,
                                                       int nx, int ny, int nz, int xcd_chunk, int bands) {
    const int N = nx * ny * nz;
    const int n = bands > 0 ? band_node(nx, ny, nz, bands, false) : node_index(xcd_chunk, N);
    if (n < 0) return;
    const int x = n % nx, t = n / nx, y = t % ny, z = t / ny;
    mh[n] = neg_lap_iso<LAT>([&](int dx, int dy, int dz) {
        return phi[wrap2(x + dx, nx) + nx * (wrap2(y + dy, ny) + ny * wrap2(z + dz, nz))];
    });
}

template <int LAT, int NC, typename P, bool MRT, bool ISO>
__global__ __launch_bounds__(256) void k_collide_stream(KParams kp, const P* __restrict__ g,
                                                        P* __restrict__ gn,
                                                        const float* __restrict__ rref,
                                                        const double* __restrict__ rt,
                                                        const double* __restrict__ lnf,
                                                        const P* fsum_in, P* fsum_out, int xcd_chunk, int nt,
                                                        int rev, int zs, int bands) {
    const int n = bands > 0 ? band_node(kp.nx, kp.ny, kp.nz, bands, rev != 0)
                            : slab_order(node_index(xcd_chunk, kp.N, rev != 0), kp.nx, kp.ny, kp.nz, zs);
    if (n < 0) return;
    const Dims dm{kp.nx, kp.ny, kp.nz, kp.N};
    node_collide_stream<LAT, NC, P, MRT, true, ISO>(kp, dm, n, g, gn, rref, rt, lnf, fsum_in, fsum_out, nt != 0);
}

// ------------------------------------------------ steps 6-9, z-marching form
// D3Q19.  A 256-thread workgroup owns a kZX x kZY tile of (x, y) and sweeps the
// planes z0 .. z1-1 of its z-range.  The FP64 fields of the moments pass are
// staged through LDS so that each is read from memory about once per step
// instead of once per stencil point:
//   phi        planes z-1, z, z+1 (tile + halo 2) in a ring of 4 slots, while
//              plane z+2 is loaded into the fourth;
//   rt, ln f   plane z (tile + halo 1) in a ring of 2 slots, while plane z+1 is
//              loaded into the other;
// the node's own column supplies phi(z-2) and rt, ln f(z-1) from registers
// (values of earlier planes) and phi(z+2), rt, ln f(z+1) from registers loaded
// one plane early, together with the node's populations.  The per-node
// arithmetic is stencil_force + collide_push_loaded, as in k_collide_stream.
constexpr int kZX = 64, kZY = 4;
constexpr int kPhiW = kZX + 4, kPhiH = kZY + 4;  // phi tile + halo 2
constexpr int kRlW = kZX + 2, kRlH = kZY + 2;    // rt / ln f tile + halo 1
constexpr int kPhiPts = kPhiW * kPhiH;
constexpr int kRlPts = kRlW * kRlH;
constexpr int kPhiPer = (kPhiPts + 255) / 256;   // fill points per thread
constexpr int kRlPer = (kRlPts + 255) / 256;

// Waves per SIMD the z-marching kernel is compiled for: two (at most 256
// registers per lane) for FP32 populations with one or two components, where
// the MRT collision would otherwise take a few more and halve the occupancy;
// the compiler's choice otherwise.
template <int NC, typename P>
constexpr int kZmarchWaves = (sizeof(P) == 4 && NC <= 2) ? 2 : 1;

// The tile (txy) and z-range (zc) of z-marching workgroup b, or false for a
// workgroup with no work.  Hardware block b runs on XCD b % 8.
//   zorder 0: XCD-contiguous chunks: XCD k takes the logical blocks
//             k * xcd_chunk .. (k + 1) * xcd_chunk - 1 (tiles fastest, then
//             z-ranges; xcd_chunk = 0: logical block b);
//   zorder 1: XCD y-bands: the tile rows are cut into 8 bands of at most
//             ceil(tiles_y / 8) rows, XCD k takes band k of every z-range,
//             z-ranges in order, so that all XCDs march through the same planes
//             at once (the DRAM pages of every stream then open for one window
//             of addresses instead of eight) and a band's halo planes, read
//             again by its next z-range, stay in its XCD's L2.  The grid is
//             zmarch_grid() blocks; a shorter band leaves blocks idle.
__device__ __forceinline__ bool zmarch_tile_of_block(int b, int tiles_x, int tiles_y, int nzc, int xcd_chunk,
                                                     int zorder, int& zc, int& txy) {
    if (zorder == 1) {
        const int k = b & 7, j = b >> 3;
        const int rows = (tiles_y + 7) >> 3;           // tile rows per band, at most
        const int per = rows * tiles_x;                 // blocks per band and z-range
        zc = j / per;
        const int tl = j - zc * per;
        const int r0 = (k * tiles_y) >> 3, r1 = ((k + 1) * tiles_y) >> 3;
        const int ty = r0 + tl / tiles_x;
        txy = ty * tiles_x + tl % tiles_x;
        return zc < nzc && ty < r1;
    }
    const int lb = xcd_chunk > 0 ? (b & 7) * xcd_chunk + (b >> 3) : b;
    zc = lb / (tiles_x * tiles_y);
    txy = lb - zc * tiles_x * tiles_y;
    return lb < tiles_x * tiles_y * nzc;
}

template <int NC, typename P, bool MRT, int DIR>
__global__ __launch_bounds__(256, (kZmarchWaves<NC, P>)) void k_collide_zmarch(KParams kp, const P* __restrict__ g,
                                                        P* __restrict__ gn,
                                                        const float* __restrict__ rref,
                                                        const double* __restrict__ rt,
                                                        const double* __restrict__ lnf,
                                                        const P* fsum_in, P* fsum_out, int zlen, int xcd_chunk,
                                                        int nt, int zorder) {
    // DIR = +1 marches each z-range upward, -1 downward (and takes an XCD's
    // z-ranges top-down), so that a pass following one sweep starts where that
    // sweep ended.  All ring bookkeeping is relative to the march direction:
    // "ahead" is z + DIR.
    static_assert(DIR == 1 || DIR == -1, "march direction");
    const int nx = kp.nx, ny = kp.ny, nz = kp.nz;
    const size_t N = kp.N;
    const int plane = nx * ny;
    const int tiles_x = nx / kZX;
    const int tiles_xy = tiles_x * (ny / kZY);
    const int nzc = (nz + zlen - 1) / zlen;
    const int b = blockIdx.x;
    int zc, txy;
    if (zorder == 1) {
        // XCD y-bands (z-ranges top-down when marching downward)
        if (!zmarch_tile_of_block(b, tiles_x, tiles_xy / tiles_x, nzc, 0, 1, zc, txy)) return;
        if (DIR < 0) zc = nzc - 1 - zc;
    } else {
        const int j = b >> 3;
        const int lb = xcd_chunk > 0 ? (b & 7) * xcd_chunk + (DIR > 0 ? j : xcd_chunk - 1 - j) : b;
        if (lb >= tiles_xy * nzc) return;  // whole workgroup, before any barrier
        zc = lb / tiles_xy;
        txy = lb - zc * tiles_xy;
    }
    const int x0 = (txy % tiles_x) * kZX, y0 = (txy / tiles_x) * kZY;
    const int z0 = zc * zlen, z1 = min(z0 + zlen, nz);
    const int start = DIR > 0 ? z0 : z1 - 1;
    const int t = threadIdx.x;
    const int tx = t % kZX, ty = t / kZX;
    const int x = x0 + tx, y = y0 + ty;
    const int col = x + nx * y;
    const Dims dm{nx, ny, nz, kp.N};
    const double* phig = lnf + (size_t)NC * N;

    __shared__ double s_phi[4][kPhiPts];
    __shared__ double s_rl[2][2 * NC][kRlPts];  // rt_i, then ln f_i

    // fill pattern, the same for every plane: byte offset of each point in its
    // plane (points past the tile read offset 0 and are not stored)
    unsigned phi_off[kPhiPer], rl_off[kRlPer];
#pragma unroll
    for (int k = 0; k < kPhiPer; ++k) {
        const int p = t + 256 * k;
        phi_off[k] = p < kPhiPts ? 8u * (unsigned)(wrap2(x0 - 2 + p % kPhiW, nx) + nx * wrap2(y0 - 2 + p / kPhiW, ny)) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kRlPer; ++k) {
        const int p = t + 256 * k;
        rl_off[k] = p < kRlPts ? 8u * (unsigned)(wrap2(x0 - 1 + p % kRlW, nx) + nx * wrap2(y0 - 1 + p / kRlW, ny)) : 0u;
    }
    // only the last fill row can run past the tile
    auto phi_fills = [&](int k) { return k < kPhiPer - 1 || t + 256 * k < kPhiPts; };
    auto rl_fills = [&](int k) { return k < kRlPer - 1 || t + 256 * k < kRlPts; };
    auto zoff = [&](int zz) { return (size_t)wrap2(zz, nz) * plane; };
    auto rl_src = [&](int f) { return f < NC ? rt + (size_t)f * N : lnf + (size_t)(f - NC) * N; };
    const unsigned col8 = 8u * (unsigned)col;

    // prologue: phi planes start - DIR, start, start + DIR -> slots 0, 1, 2;
    // rt / ln f plane start -> slot 0; the own column's planes behind in registers
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double* src = phig + zoff(start + (d - 1) * DIR);
#pragma unroll
        for (int k = 0; k < kPhiPer; ++k)
            if (phi_fills(k)) s_phi[d][t + 256 * k] = ld(src, phi_off[k]);
    }
#pragma unroll
    for (int f = 0; f < 2 * NC; ++f) {
        const double* src = rl_src(f) + zoff(start);
#pragma unroll
        for (int k = 0; k < kRlPer; ++k)
            if (rl_fills(k)) s_rl[0][f][t + 256 * k] = ld(src, rl_off[k]);
    }
    double phi_b2 = ld(phig + zoff(start - 2 * DIR), col8);
    double phi_b1 = ld(phig + zoff(start - DIR), col8);
    double rl_b1[2 * NC];
#pragma unroll
    for (int f = 0; f < 2 * NC; ++f) rl_b1[f] = ld(rl_src(f) + zoff(start - DIR), col8);
    // The node's inputs and its own column ahead (phi two planes, rt / ln f one
    // plane along the march) are loaded one plane early, the first here: their
    // latency overlaps the barrier and the ring stores instead of the stencil.
    NodeIn<1, NC, P> in;
    load_node_inputs<1, NC, P, true>(g, fsum_in, rref, col + start * plane, N, in);
    double phi_a2 = ld(phig + zoff(start + 2 * DIR), col8);
    double rl_a1[2 * NC];
#pragma unroll
    for (int f = 0; f < 2 * NC; ++f) rl_a1[f] = ld(rl_src(f) + zoff(start + DIR), col8);
    __syncthreads();

    const int cphi = (ty + 2) * kPhiW + tx + 2;  // this node in the phi tile
    const int crl = (ty + 1) * kRlW + tx + 1;    // this node in the rt / ln f tile
    for (int it = 0; it < z1 - z0; ++it) {
        const int zz = start + it * DIR;
        // loads of the planes being filled (written to LDS after the node's work)
        double fphi[kPhiPer], frl[2 * NC][kRlPer];
        const double* phi2 = phig + zoff(zz + 2 * DIR);
#pragma unroll
        for (int k = 0; k < kPhiPer; ++k) fphi[k] = ld(phi2, phi_off[k]);
        const size_t a1off = zoff(zz + DIR);
#pragma unroll
        for (int f = 0; f < 2 * NC; ++f)
#pragma unroll
            for (int k = 0; k < kRlPer; ++k) frl[f][k] = ld(rl_src(f) + a1off, rl_off[k]);
        // keep these fill loads ahead of the node's work (the scheduler would
        // otherwise sink them next to their use at the end of the iteration)
        __builtin_amdgcn_sched_barrier(0);

        // plane start + (j - 1) DIR lives in phi slot j & 3, plane start + j DIR
        // in rt / ln f slot j & 1
        const int s0 = (it + 1) & 3;
        const int r0 = it & 1;
        auto phi_at = [&](int dx, int dy, int dz) -> double {
            const int d = dz * DIR;  // offset along the march
            if (d == -2) return phi_b2;
            if (d == 2) return phi_a2;
            return s_phi[(s0 + d) & 3][cphi + dy * kPhiW + dx];
        };
        auto rl_at = [&](int f, int dx, int dy, int dz) -> double {
            const int d = dz * DIR;
            if (d == -1) return rl_b1[f];
            if (d == 1) return rl_a1[f];
            return s_rl[r0][f][crl + dy * kRlW + dx];
        };
        P F[NC][3], G[NC][3];
        double Fs[3];
        stencil_force<3, NC, P>(
            kp, phi_at, [&](int i, int dx, int dy, int dz) { return rl_at(i, dx, dy, dz); },
            [&](int i, int dx, int dy, int dz) { return rl_at(NC + i, dx, dy, dz); }, F, G, Fs);
        collide_push_loaded<1, NC, P, MRT>(kp, dm, col + zz * plane, x, y, zz, in, gn, F, G, Fs, fsum_out,
                                           nt != 0);
        if (it + 1 < z1 - z0) {  // the next plane's inputs
            load_node_inputs<1, NC, P, true>(g, fsum_in, rref, col + (zz + DIR) * plane, N, in);
            phi_a2 = ld(phig + zoff(zz + 3 * DIR), col8);
#pragma unroll
            for (int f = 0; f < 2 * NC; ++f) rl_a1[f] = ld(rl_src(f) + zoff(zz + 2 * DIR), col8);
        }

        // shift the own-column registers, store the filled planes, publish
        phi_b2 = phi_b1;
        phi_b1 = s_phi[s0][cphi];
#pragma unroll
        for (int f = 0; f < 2 * NC; ++f) rl_b1[f] = s_rl[r0][f][crl];
#pragma unroll
        for (int k = 0; k < kPhiPer; ++k)
            if (phi_fills(k)) s_phi[(it + 3) & 3][t + 256 * k] = fphi[k];
#pragma unroll
        for (int f = 0; f < 2 * NC; ++f)
#pragma unroll
            for (int k = 0; k < kRlPer; ++k)
                if (rl_fills(k)) s_rl[(it + 1) & 1][f][t + 256 * k] = frl[f][k];
        __syncthreads();
    }
}

// ------------------------- steps 6-9, z-marching form, isotropic stencils
// D3Q19.  A 256-thread workgroup owns a kZX x kZY tile of (x, y) and sweeps the
// planes z0 .. z1-1 of its z-range upward; no Laplacian pass runs before it.
// LDS holds
//   phi          four planes (tile + halo 2) in a ring;
//   mu_i, rho~_i three planes (tile + halo 1) in three buffers, plane q in
//                buffer q mod 3: mu_i = RT ln f_i + sqrt(kappa_i) (-lap(phi))
//                is formed as a plane is filled, -lap(phi) from the phi ring.
// Node z reads mu_i and rho~_i of planes z-1, z, z+1 from LDS with the
// stencil of the one-thread-per-node kernel (stencil_force_iso_mu), so the
// result is the same bit for bit.  Per node plane z, two barriers: after the
// stencil reads (plane z-1's buffer is then refilled with plane z+2, and the
// phi slot of plane z with plane z+4), and at the end.  Planes z0-1 .. z1 of
// mu_i and rho~_i and z0-2 .. z1+1 of phi pass through a workgroup.  With
// two or three components the collision alone needs nearly all of 256
// registers, so the kernel runs at one wave per SIMD there (at two, 150
// registers spilled to scratch memory and the pass took 3.4 times as long on
// the 256^3 ternary lattice); a fourth plane buffer removing the first
// barrier, with the next plane's node inputs loaded across the second,
// measured slower (2.72 against 2.60 ms).
template <int NC, typename P>
constexpr int kZmarchIsoWaves = (sizeof(P) == 4 && NC == 1) ? 2 : 1;

__device__ __forceinline__ int mod3(int q) { return ((q % 3) + 3) % 3; }


template <int NC, typename P, bool MRT>
__global__ __launch_bounds__(256, (kZmarchIsoWaves<NC, P>)) void k_collide_zmarch_iso(
    KParams kp, const P* __restrict__ g, P* __restrict__ gn, const float* __restrict__ rref,
    const double* __restrict__ rt, const double* __restrict__ lnf, const P* fsum_in, P* fsum_out, int zlen,
    int xcd_chunk, int nt, int zorder) {
    constexpr int NF = 2 * NC;  // fields: mu_i, then rho~_i
    const int nx = kp.nx, ny = kp.ny, nz = kp.nz;
    const size_t N = kp.N;
    const int plane = nx * ny;
    const int tiles_x = nx / kZX;
    const int tiles_xy = tiles_x * (ny / kZY);
    const int nzc = (nz + zlen - 1) / zlen;
    int zc, txy;
    if (!zmarch_tile_of_block(blockIdx.x, tiles_x, tiles_xy / tiles_x, nzc, xcd_chunk, zorder, zc, txy))
        return;  // whole workgroup, before any barrier
    const int x0 = (txy % tiles_x) * kZX, y0 = (txy / tiles_x) * kZY;
    const int z0 = zc * zlen, z1 = min(z0 + zlen, nz);
    const int t = threadIdx.x;
    const int tx = t % kZX, ty = t / kZX;
    const int x = x0 + tx, y = y0 + ty;
    const int col = x + nx * y;
    const Dims dm{nx, ny, nz, kp.N};
    const double* phig = lnf + (size_t)NC * N;

    __shared__ double s_phi[4][kPhiPts];   // phi plane q in slot q & 3
    __shared__ double s_f[3][NF][kRlPts];  // mu_i, rho~_i of plane q in buffer q mod 3

    // fill pattern, the same for every plane (points past the box read offset 0
    // and are not stored)
    unsigned phi_off[kPhiPer], rl_off[kRlPer];
#pragma unroll
    for (int k = 0; k < kPhiPer; ++k) {
        const int q = t + 256 * k;
        phi_off[k] = q < kPhiPts ? 8u * (unsigned)(wrap2(x0 - 2 + q % kPhiW, nx) + nx * wrap2(y0 - 2 + q / kPhiW, ny)) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kRlPer; ++k) {
        const int q = t + 256 * k;
        rl_off[k] = q < kRlPts ? 8u * (unsigned)(wrap2(x0 - 1 + q % kRlW, nx) + nx * wrap2(y0 - 1 + q / kRlW, ny)) : 0u;
    }
    auto phi_fills = [&](int k) { return k < kPhiPer - 1 || t + 256 * k < kPhiPts; };
    auto rl_fills = [&](int k) { return k < kRlPer - 1 || t + 256 * k < kRlPts; };
    auto zoff = [&](int zz) { return (size_t)wrap2(zz, nz) * plane; };
    // ln f_i (f < NC) and rho~_i (f >= NC) of the moments pass
    auto src_of = [&](int f) { return f < NC ? lnf + (size_t)f * N : rt + (size_t)(f - NC) * N; };

    auto load_phi = [&](int q, double (&v)[kPhiPer]) {
        const double* src = phig + zoff(q);
#pragma unroll
        for (int k = 0; k < kPhiPer; ++k) v[k] = ld(src, phi_off[k]);
    };
    auto store_phi = [&](int q, const double (&v)[kPhiPer]) {
#pragma unroll
        for (int k = 0; k < kPhiPer; ++k)
            if (phi_fills(k)) s_phi[q & 3][t + 256 * k] = v[k];
    };
    // ln f_i and rho~_i of plane q at this thread's fill points
    auto load_fill = [&](int q, double (&v)[NF][kRlPer]) {
        const size_t zo = zoff(q);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < kRlPer; ++k) v[f][k] = ld(src_of(f) + zo, rl_off[k]);
    };
    // mu_i and rho~_i of plane q into its buffer (phi planes q-1 .. q+1 in the ring)
    auto store_fill = [&](int q, const double (&v)[NF][kRlPer]) {
        const int bq = mod3(q);
#pragma unroll
        for (int k = 0; k < kRlPer; ++k) {
            if (!rl_fills(k)) continue;
            const int pt = t + 256 * k;
            const int bx = pt % kRlW + 1, by = pt / kRlW + 1;  // in the phi box
            const double mh = neg_lap_iso<1>([&](int dx, int dy, int dz) {
                return s_phi[(q + dz) & 3][(by + dy) * kPhiW + bx + dx];
            });
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                s_f[bq][i][pt] = chem_pot(kp, i, v[i][k], mh);
                s_f[bq][NC + i][pt] = v[NC + i][k];
            }
        }
    };

    // prologue: phi planes z0-2 .. z0+1; mu_i, rho~_i of planes z0-1 and z0;
    // phi planes z0+2, z0+3 into the slots of z0-2, z0-1; then plane z0+1
    {
        double v[NF][kRlPer], w[NF][kRlPer], fp[kPhiPer];
#pragma unroll
        for (int d = -2; d <= 1; ++d) {
            load_phi(z0 + d, fp);
            store_phi(z0 + d, fp);
        }
        load_fill(z0 - 1, v);
        load_fill(z0, w);
        __syncthreads();
        store_fill(z0 - 1, v);
        store_fill(z0, w);
        load_fill(z0 + 1, v);
        __syncthreads();
        load_phi(z0 + 2, fp);
        store_phi(z0 + 2, fp);
        load_phi(z0 + 3, fp);
        store_phi(z0 + 3, fp);
        __syncthreads();
        store_fill(z0 + 1, v);
        __syncthreads();
    }

    const int cown = (ty + 1) * kRlW + tx + 1;
    for (int z = z0; z < z1; ++z) {
        const bool fill = z + 2 <= z1;   // plane z+2 is needed (by node z+1)
        const bool ring = z + 3 <= z1;   // phi plane z+4 is needed (for plane z+3)
        // loads first: plane z+2's fields, phi plane z+4 (their latency
        // overlaps the stencil)
        double v[NF][kRlPer], fp[kPhiPer];
        if (fill) load_fill(z + 2, v);
        if (ring) load_phi(z + 4, fp);
        __builtin_amdgcn_sched_barrier(0);

        // node z's stencil: mu_i and rho~_i of planes z-1, z, z+1
        P F[NC][3], G[NC][3];
        double Fs[3];
        const int bm = mod3(z - 1), b0 = mod3(z), bp = mod3(z + 1);
        auto buf = [&](int dz) { return dz < 0 ? bm : (dz > 0 ? bp : b0); };
        stencil_force_iso_mu<NC, P, true>(
            kp, [&](int i, int dx, int dy, int dz) { return s_f[buf(dz)][i][cown + dy * kRlW + dx]; },
            [&](int i, int dx, int dy, int dz) { return s_f[buf(dz)][NC + i][cown + dy * kRlW + dx]; }, F, G,
            Fs);
        // node z's inputs (their latency overlaps the barrier and the fill)
        NodeIn<1, NC, P> in;
        load_node_inputs<1, NC, P, true>(g, fsum_in, rref, col + z * plane, N, in);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();  // plane z-1's buffer and phi slot z are free

        collide_push_loaded<1, NC, P, MRT>(kp, dm, col + z * plane, x, y, z, in, gn, F, G, Fs, fsum_out, nt != 0);
        // the plane fills after the pushes: the stores drain while the
        // Laplacians and chemical potentials are formed
        if (fill) store_fill(z + 2, v);
        if (ring) store_phi(z + 4, fp);
        __syncthreads();
    }
}

// ------------- steps 6-9, z-marching form, isotropic stencils, one component per thread group
// The same tile, rings and stencil as k_collide_zmarch_iso, for the
// component-major layout (N_c >= 3), with the work of a node split by
// component: the workgroup has N_c groups of 256 threads and group c owns
// component c of every node of the tile.  A group reads its component's Q
// population streams, forms mu_c and rho~_c of the planes it fills, the
// stencil and force of component c, its density and momentum, and collides
// and pushes component c.  The velocity needs every component's density and
// momentum and the force sum every component's force: each group writes its
// seven FP64 values per node to LDS before the first barrier of a plane and
// reads the others' after it, summing in component order, so the result is
// the same bit for bit as the kernels that keep a node in one thread.  A
// thread then holds one component's collision instead of N_c: at three
// components 768 threads, three waves per SIMD, where the one-thread-per-node
// z-march needs more than 256 registers per lane and runs one.
template <int NC, typename P, bool MRT>
__global__ __launch_bounds__(256 * NC) void k_collide_zmarch_iso_cs(
    KParams kp, const P* __restrict__ g, P* __restrict__ gn, const float* __restrict__ rref,
    const double* __restrict__ rt, const double* __restrict__ lnf, const P* fsum_in, P* fsum_out, int zlen,
    int xcd_chunk, int nt, int zorder) {
    static_assert(!kInterleaved<NC>, "component-major layout only");
    static_assert(kPhiPts <= 256 * NC, "one phi fill point per thread");
    using L = Lat<1>;
    constexpr int Q = L::Q;
    constexpr int kX = 7;  // exchanged per node and component: rho, j (3), f (3)
    const int nx = kp.nx, ny = kp.ny, nz = kp.nz;
    const size_t N = kp.N;
    const int plane = nx * ny;
    const int tiles_x = nx / kZX;
    const int tiles_xy = tiles_x * (ny / kZY);
    const int nzc = (nz + zlen - 1) / zlen;
    int zc, txy;
    if (!zmarch_tile_of_block(blockIdx.x, tiles_x, tiles_xy / tiles_x, nzc, xcd_chunk, zorder, zc, txy))
        return;  // whole workgroup, before any barrier
    const int x0 = (txy % tiles_x) * kZX, y0 = (txy / tiles_x) * kZY;
    const int z0 = zc * zlen, z1 = min(z0 + zlen, nz);
    const int tg = threadIdx.x;
    // this thread's component: uniform over a wave (256 is a multiple of 64),
    // taken into a scalar register so that its addresses are scalar too
    const int c = __builtin_amdgcn_readfirstlane(tg >> 8);
    const int t = tg & 255;      // this thread's node in the tile
    const int tx = t % kZX, ty = t / kZX;
    const int x = x0 + tx, y = y0 + ty;
    const int col = x + nx * y;
    const Dims dm{nx, ny, nz, kp.N};
    const double* phig = lnf + (size_t)NC * N;
    const double* lnf_c = lnf + (size_t)c * N;
    const double* rt_c = rt + (size_t)c * N;

    __shared__ double s_phi[4][kPhiPts];   // phi plane q in slot q & 3
    __shared__ double s_f[3][2 * NC][kRlPts];  // mu_i, rho~_i of plane q in buffer q mod 3
    __shared__ double s_x[NC][kX][256];    // per-node exchange between the groups

    // fill pattern: one phi point per thread (the whole workgroup), and
    // kRlPer points of its own component's mu and rho~ per thread of a group
    const bool phi_fill = tg < kPhiPts;
    const unsigned phi_off =
        phi_fill ? 8u * (unsigned)(wrap2(x0 - 2 + tg % kPhiW, nx) + nx * wrap2(y0 - 2 + tg / kPhiW, ny)) : 0u;
    unsigned rl_off[kRlPer];
#pragma unroll
    for (int k = 0; k < kRlPer; ++k) {
        const int q = t + 256 * k;
        rl_off[k] = q < kRlPts ? 8u * (unsigned)(wrap2(x0 - 1 + q % kRlW, nx) + nx * wrap2(y0 - 1 + q / kRlW, ny)) : 0u;
    }
    auto rl_fills = [&](int k) { return k < kRlPer - 1 || t + 256 * k < kRlPts; };
    auto zoff = [&](int zz) { return (size_t)wrap2(zz, nz) * plane; };
    auto load_phi = [&](int q) { return ld(phig + zoff(q), phi_off); };
    auto store_phi = [&](int q, double v) {
        if (phi_fill) s_phi[q & 3][tg] = v;
    };
    // ln f_c and rho~_c of plane q at this thread's fill points
    auto load_fill = [&](int q, double (&v)[2][kRlPer]) {
        const size_t zo = zoff(q);
#pragma unroll
        for (int k = 0; k < kRlPer; ++k) {
            v[0][k] = ld(lnf_c + zo, rl_off[k]);
            v[1][k] = ld(rt_c + zo, rl_off[k]);
        }
    };
    // mu_c and rho~_c of plane q into its buffer (phi planes q-1 .. q+1 in the ring)
    auto store_fill = [&](int q, const double (&v)[2][kRlPer]) {
        const int bq = mod3(q);
#pragma unroll
        for (int k = 0; k < kRlPer; ++k) {
            if (!rl_fills(k)) continue;
            const int pt = t + 256 * k;
            const int bx = pt % kRlW + 1, by = pt / kRlW + 1;  // in the phi box
            const double mh = neg_lap_iso<1>([&](int dx, int dy, int dz) {
                return s_phi[(q + dz) & 3][(by + dy) * kPhiW + bx + dx];
            });
            s_f[bq][c][pt] = chem_pot(kp, c, v[0][k], mh);
            s_f[bq][NC + c][pt] = v[1][k];
        }
    };
    // component c's inputs of node plane zz: populations, rest reference, the
    // previous step's force sum
    P gv[Q], fprev[3];
    float ref = 0.f;
    auto load_inputs = [&](int zz) {
        const int n = col + zz * plane;
        const unsigned off = pop_off<NC, P>(n);
#pragma unroll
        for (int k = 0; k < 3; ++k) fprev[k] = ld(fsum_in, ((unsigned)n * 3 + k) * (unsigned)sizeof(P));
#pragma unroll
        for (int a = 0; a < Q; ++a)
            gv[a] = __builtin_nontemporal_load(reinterpret_cast<const P*>(
                reinterpret_cast<const char*>(pop_base<NC, Q>(g, c, a, N)) + off));
        if constexpr (sizeof(P) == 4) ref = ld(rref, ((unsigned)n * NC + c) * 4u);
    };

    // prologue, as in k_collide_zmarch_iso
    {
        double v[2][kRlPer], w[2][kRlPer];
#pragma unroll
        for (int d = -2; d <= 1; ++d) store_phi(z0 + d, load_phi(z0 + d));
        load_fill(z0 - 1, v);
        load_fill(z0, w);
        __syncthreads();
        store_fill(z0 - 1, v);
        store_fill(z0, w);
        load_fill(z0 + 1, v);
        __syncthreads();
        store_phi(z0 + 2, load_phi(z0 + 2));
        store_phi(z0 + 3, load_phi(z0 + 3));
        __syncthreads();
        store_fill(z0 + 1, v);
        load_inputs(z0);
        __syncthreads();
    }

    const int cown = (ty + 1) * kRlW + tx + 1;
    for (int z = z0; z < z1; ++z) {
        const bool fill = z + 2 <= z1;   // plane z+2 is needed (by node z+1)
        const bool ring = z + 3 <= z1;   // phi plane z+4 is needed (for plane z+3)
        double v[2][kRlPer], fp = 0.0;
        if (fill) load_fill(z + 2, v);
        if (ring) fp = load_phi(z + 4);
        __builtin_amdgcn_sched_barrier(0);

        // component c's stencil at node z: mu_c and rho~_c of planes z-1, z, z+1
        const int bm = mod3(z - 1), b0 = mod3(z), bp = mod3(z + 1);
        auto buf = [&](int dz) { return dz < 0 ? bm : (dz > 0 ? bp : b0); };
        double gmu[3], grt[3];
        double rc;
        {
            auto mu = [&](int dz) {
                return [&, dz](int dx, int dy) { return s_f[buf(dz)][c][cown + dy * kRlW + dx]; };
            };
            auto r = [&](int dz) {
                return [&, dz](int dx, int dy) { return s_f[buf(dz)][NC + c][cown + dy * kRlW + dx]; };
            };
            const IsoCross mdn = iso_cross(mu(-1)), mup = iso_cross(mu(1));
            const IsoOwn mown = iso_own(mu(0));
            iso_grad(mown.sx + mdn.ax, mown.sy + mdn.ay, mdn.b, mup, gmu);
            const IsoCross rdn = iso_cross(r(-1)), rup = iso_cross(r(1));
            const IsoOwn rown = iso_own(r(0));
            iso_grad(rown.sx + rdn.ax, rown.sy + rdn.ay, rdn.b, rup, grt);
            rc = rown.c;
        }
        double f[3];
        P F[3], G[3];
        comp_force<P>(kp, c, gmu, grt, rc, f, F, G);
        // component c's density and momentum
        double rho, mov, jc[3];
        comp_density<L, P>(gv, ref, rho, mov);
        comp_momentum<L, P>(gv, jc);
        s_x[c][0][t] = rho;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_x[c][1 + k][t] = jc[k];
            s_x[c][4 + k][t] = f[k];
        }
        __syncthreads();  // stencil reads of plane z-1's buffer done; exchange visible

        // totals in component order (as collide_push_loaded sums them)
        double rtot = 0.0, j[3] = {0.0, 0.0, 0.0}, Fs[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            rtot += s_x[i][0][t];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                j[k] += s_x[i][1 + k][t];
                Fs[k] += s_x[i][4 + k][t];
            }
        }
        double u[3];
        node_velocity<3, P>(kp, rtot, j, Fs, fprev, u);
        const int n = col + z * plane;
        P oc[Q];
        collide_comp<L, P, MRT, kPairCollision<NC, P>>(kp, gv, rho, mov, u, F, G, oc);
        push_comp<L, NC, P>(PushGeom<3, NC, P>(dm, n, x, y, z), gn, c, N, oc, nt != 0);
        if (c == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) st(fsum_out, ((unsigned)n * 3 + k) * (unsigned)sizeof(P), (P)Fs[k]);
        }
        if (z + 1 < z1) load_inputs(z + 1);
        // the plane fills after the pushes and the next plane's loads: the
        // stores drain and the loads arrive while the Laplacians are formed
        if (fill) store_fill(z + 2, v);
        if (ring) store_phi(z + 4, fp);
        __syncthreads();  // fills of planes z+2 / z+4 visible; exchange free
    }
}

// ------------------------------------------------------------ initial state
// g = g_eq(rho_i, u) (eq. eqLBEMCb), zero force history.
template <int LAT, int NC, typename P>
__global__ __launch_bounds__(256) void k_init(KParams kp, const double* __restrict__ rho_molar,
                                              const double* __restrict__ uin, P* __restrict__ g,
                                              float* __restrict__ rref, P* __restrict__ fsum) {
    using L = Lat<LAT>;
    constexpr int D = L::D, Q = L::Q;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= kp.N) return;
    const size_t N = kp.N;
    double u[3] = {0.0, 0.0, 0.0};
    if (uin)
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = uin[(size_t)k * N + n];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double rho = rho_molar[(size_t)c * N + n] * kp.M[c];
        double ref = 0.0;
        if constexpr (sizeof(P) == 4) {
            const float rf = (float)rho;
            rref[(size_t)n * NC + c] = rf;
            ref = (double)rf;
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const double eu = L::ex[a] * u[0] + L::ey[a] * u[1] + L::ez[a] * u[2];
            double ge = L::w[a] * rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
            if (kp.standard)
                ge += L::w[a] * rho;  // standard equilibrium w_a rho (1 + ...)
            else if (a == 0)
                ge += rho - ref;
            g[pop_index<NC, Q>(c, a, n, N)] = (P)ge;
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) fsum[(size_t)n * D + k] = (P)0;
}

// ------------------------------------------------------------ output fields
template <int LAT, int NC, typename P>
__global__ __launch_bounds__(256) void k_fields(KParams kp, const P* __restrict__ g,
                                                const float* __restrict__ rref,
                                                const P* __restrict__ fsum,
                                                double* __restrict__ rho_molar, double* __restrict__ uout,
                                                double* __restrict__ pout, double* __restrict__ lnf) {
    using L = Lat<LAT>;
    constexpr int D = L::D, Q = L::Q;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= kp.N) return;
    const size_t N = kp.N;
    P gv[NC][Q];
    load_pops<L, NC, P>(g, n, N, gv);
    double rho[NC], mov[NC], r[NC], lf[NC];
    densities<L, NC, P>(gv, rref, n, N, rho, mov);
    double rtot = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        r[c] = rho[c] / kp.M[c];
        rho_molar[(size_t)c * N + n] = r[c];
        rtot += rho[c];
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            j[0] += (double)gv[c][a] * L::ex[a];
            j[1] += (double)gv[c][a] * L::ey[a];
            j[2] += (double)gv[c][a] * L::ez[a];
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) uout[(size_t)k * N + n] = (j[k] + 0.5 * (double)fsum[(size_t)n * D + k]) / rtot;
    double p;
    eos_lnf<NC>(kp, r, lf, &p);
    pout[n] = p;
#pragma unroll
    for (int c = 0; c < NC; ++c) lnf[(size_t)c * N + n] = lf[c];
}

// Populations as FP64 [c][a][n] (rest slot with its reference added back).
template <int LAT, int NC, typename P>
__global__ __launch_bounds__(256) void k_export_pops(KParams kp, const P* __restrict__ g,
                                                     const float* __restrict__ rref, double* __restrict__ out) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= kp.N) return;
    const size_t N = kp.N;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < L::Q; ++a) {
            double v = (double)g[pop_index<NC, L::Q>(c, a, n, N)];
            if constexpr (sizeof(P) == 4)
                if (a == 0) v += (double)rref[(size_t)n * NC + c];
            out[(size_t)(c * L::Q + a) * N + n] = v;
        }
}

// ---------------------------------------------------------------- reductions
// Block-level deterministic reduction: each block writes NC partial sums of
// rho_i (mass) and, when snap != nullptr, NC maxima of |rho_i - snap_i| and of
// rho_i, then updates the snapshot.  A single-block pass combines partials in
// block order.
constexpr int kRedBlock = 256;

template <int LAT, int NC, typename P>
__global__ __launch_bounds__(kRedBlock) void k_reduce_partials(KParams kp, const P* __restrict__ g,
                                                               const float* __restrict__ rref,
                                                               double* __restrict__ snap,
                                                               double* __restrict__ partial) {
    using L = Lat<LAT>;
    __shared__ double sh[3 * NC][kRedBlock];
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = kp.N;
    double rho[NC] = {}, dif[NC] = {}, mx[NC] = {};
    if (n < kp.N) {
        P gv[NC][L::Q];
        load_pops<L, NC, P>(g, n, N, gv);
        double mov[NC];
        densities<L, NC, P>(gv, rref, n, N, rho, mov);
        if (snap) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double old = snap[(size_t)c * N + n];
                dif[c] = fabs(rho[c] - old);
                mx[c] = fabs(rho[c]);
                snap[(size_t)c * N + n] = rho[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        sh[c][threadIdx.x] = rho[c];
        sh[NC + c][threadIdx.x] = dif[c];
        sh[2 * NC + c][threadIdx.x] = mx[c];
    }
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
                sh[NC + c][threadIdx.x] = fmax(sh[NC + c][threadIdx.x], sh[NC + c][threadIdx.x + s]);
                sh[2 * NC + c][threadIdx.x] = fmax(sh[2 * NC + c][threadIdx.x], sh[2 * NC + c][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3 * NC) partial[(size_t)blockIdx.x * 3 * NC + threadIdx.x] = sh[threadIdx.x][0];
}

template <int NC>
__global__ __launch_bounds__(kRedBlock) void k_reduce_final(const double* __restrict__ partial, int nblocks,
                                                            double* __restrict__ out) {
    __shared__ double sh[3 * NC][kRedBlock];
    double acc[3 * NC] = {};
    // each thread folds a contiguous run of blocks in order
    const int per = (nblocks + kRedBlock - 1) / kRedBlock;
    const int b0 = threadIdx.x * per;
    for (int b = b0; b < b0 + per && b < nblocks; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            acc[c] += partial[(size_t)b * 3 * NC + c];
            acc[NC + c] = fmax(acc[NC + c], partial[(size_t)b * 3 * NC + NC + c]);
            acc[2 * NC + c] = fmax(acc[2 * NC + c], partial[(size_t)b * 3 * NC + 2 * NC + c]);
        }
#pragma unroll
    for (int q = 0; q < 3 * NC; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
                sh[NC + c][threadIdx.x] = fmax(sh[NC + c][threadIdx.x], sh[NC + c][threadIdx.x + s]);
                sh[2 * NC + c][threadIdx.x] = fmax(sh[2 * NC + c][threadIdx.x], sh[2 * NC + c][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3 * NC) out[threadIdx.x] = sh[threadIdx.x][0];
}

// ------------------------------------------------------------------ launchers
static inline dim3 grid_for(int N, int block) { return dim3((N + block - 1) / block); }

template <typename T>
struct Tag {
    using type = T;
};

// Calls f(lattice, components, population type) with compile-time values.
template <typename F>
void dispatch(int lattice, int nc, int precision, F&& f) {
    auto run_nc = [&](auto latc, auto ncc) {
        if (precision == 0)
            f(latc, ncc, Tag<double>{});
        else
            f(latc, ncc, Tag<float>{});
    };
    auto run_lat = [&](auto latc) {
        switch (nc) {
            case 1: run_nc(latc, std::integral_constant<int, 1>{}); break;
            case 2: run_nc(latc, std::integral_constant<int, 2>{}); break;
            case 3: run_nc(latc, std::integral_constant<int, 3>{}); break;
            default: run_nc(latc, std::integral_constant<int, 4>{}); break;
        }
    };
    if (lattice == 0)
        run_lat(std::integral_constant<int, 0>{});
    else
        run_lat(std::integral_constant<int, 1>{});
}

#define FL_TYPES                                  \
    constexpr int LAT = decltype(latc)::value;    \
    constexpr int NC = decltype(ncc)::value;      \
    using P = typename decltype(pt)::type

static inline int xcd_chunk_for(const LaunchCfg& lc, int nblocks) {
    return lc.xcd_remap ? (nblocks + 7) / 8 : 0;
}

static inline dim3 grid_remapped(int nblocks, int chunk) { return dim3(chunk > 0 ? 8 * chunk : nblocks); }

// Blocks of a z-marching launch in XCD y-band order (zmarch_tile_of_block).
static inline int zmarch_grid(int tiles_x, int tiles_y, int nzc) { return 8 * ((tiles_y + 7) / 8) * tiles_x * nzc; }

// Planes per slab of the visiting order (slab_order): one slab per XCD on a
// D3Q19 lattice when enabled, 0 (plain order) otherwise.
static inline int slab_planes(const LaunchCfg& lc, const KParams& kp) {
    return (lc.slab_order && lc.lattice == 1) ? (kp.nz + 7) / 8 : 0;
}

hipError_t launch_moments_eos(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                              double* rt, double* lnf, int* err) {
    const int bs = lc.block_k1;
    const int nb = (kp.N + bs - 1) / bs;
    const int ch = xcd_chunk_for(lc, nb);
    // two nodes per thread where the pass runs at its defaults (256-thread
    // blocks in plain block order) on an even number of FP32 nodes of >= 3
    // components; the block-size and block-order keys select the one-node form
    const bool pair = lc.mpair && lc.nc >= 3 && kp.N % 2 == 0 && bs == 256 &&
                      ch == 0 && slab_planes(lc, kp) == 0;
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        if constexpr (!kInterleaved<NC> && sizeof(P) == 4) {
            if (pair) {
                k_moments_eos_pair<LAT, NC><<<(kp.N / 2 + 255) / 256, 256, 0, lc.stream>>>(
                    kp, (const float*)g, rref, rt, lnf, err);
                return;
            }
        }
        k_moments_eos<LAT, NC, P><<<grid_remapped(nb, ch), bs, 0, lc.stream>>>(
            kp, (const P*)g, rref, rt, lnf, err, ch, slab_planes(lc, kp));
    });
    return hipGetLastError();
}

hipError_t launch_interface_lap(const LaunchCfg& lc, const KParams& kp, double* lnf) {
    const int nb = (kp.N + 255) / 256;
    const int ch = xcd_chunk_for(lc, nb);
    const int bands = lc.bands_lap;
    const dim3 grid = bands > 0 ? dim3(band_grid(kp.nx, kp.ny, kp.nz, bands, 256)) : grid_remapped(nb, ch);
    const double* phi = lnf + (size_t)lc.nc * kp.N;
    double* mh = lnf + (size_t)(lc.nc + 1) * kp.N;
    if (lc.lattice == 0)
        k_interface_lap<0><<<grid, 256, 0, lc.stream>>>(phi, mh, kp.nx, kp.ny, kp.nz, ch, bands);
    else
        k_interface_lap<1><<<grid, 256, 0, lc.stream>>>(phi, mh, kp.nx, kp.ny, kp.nz, ch, bands);
    return hipGetLastError();
}

hipError_t launch_collide_stream(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn,
                                 const float* rref, const double* rt, const double* lnf, const void* fsum_in,
                                 void* fsum_out) {
    const int bs = lc.block_k2;
    const int nb = (kp.N + bs - 1) / bs;
    const int ch = lc.xcd_remap_k2 ? xcd_chunk_for(lc, nb) : 0;
    const int nt = lc.nt_store ? 1 : 0;
    const int rev = lc.reverse_k2 ? 1 : 0;
    const int bands = lc.bands;
    const dim3 grid = bands > 0 ? dim3(band_grid(kp.nx, kp.ny, kp.nz, bands, bs)) : grid_remapped(nb, ch);
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        auto go = [&](auto mrtc, auto isoc) {
            k_collide_stream<LAT, NC, P, decltype(mrtc)::value, decltype(isoc)::value>
                <<<grid, bs, 0, lc.stream>>>(kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in,
                                             (P*)fsum_out, ch, nt, rev, slab_planes(lc, kp), bands);
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        if (lc.mrt) {
            if (kp.iso) go(T_{}, T_{}); else go(T_{}, F_{});
        } else {
            if (kp.iso) go(F_{}, T_{}); else go(F_{}, F_{});
        }
    });
    return hipGetLastError();
}

bool zmarch_fits(int lattice, int nc, int nx, int ny) {
    return lattice == 1 && nc <= 3 && nx % kZX == 0 && ny % kZY == 0;
}

hipError_t launch_collide_zmarch(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn,
                                 const float* rref, const double* rt, const double* lnf, const void* fsum_in,
                                 void* fsum_out) {
    if (!zmarch_fits(lc.lattice, lc.nc, kp.nx, kp.ny) || lc.zlen < 1) return hipErrorInvalidValue;
    const int tx = kp.nx / kZX, ty = kp.ny / kZY, nzc = (kp.nz + lc.zlen - 1) / lc.zlen;
    const int nb = tx * ty * nzc;
    const int ch = xcd_chunk_for(lc, nb);
    const int nt = lc.nt_store ? 1 : 0;
    const dim3 grid = lc.zorder == 1 ? dim3(zmarch_grid(tx, ty, nzc)) : grid_remapped(nb, ch);
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        if constexpr (LAT == 1 && NC <= 3) {
            // march downward when the passes alternate direction (reverse_k2)
            auto go = [&](auto mrt, auto dir) {
                k_collide_zmarch<NC, P, decltype(mrt)::value, decltype(dir)::value>
                    <<<grid, 256, 0, lc.stream>>>(kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in,
                                                  (P*)fsum_out, lc.zlen, ch, nt, lc.zorder);
            };
            using Up = std::integral_constant<int, 1>;
            using Down = std::integral_constant<int, -1>;
            if (lc.mrt) {
                if (lc.reverse_k2) go(std::true_type{}, Down{}); else go(std::true_type{}, Up{});
            } else {
                if (lc.reverse_k2) go(std::false_type{}, Down{}); else go(std::false_type{}, Up{});
            }
        }
    });
    return hipGetLastError();
}

hipError_t launch_collide_zmarch_iso(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn,
                                     const float* rref, const double* rt, const double* lnf, const void* fsum_in,
                                     void* fsum_out) {
    // nz >= 2: the prologue reads phi three planes above a z-range's start,
    // which wrap2 folds into [0, nz) only from two planes on
    if (!zmarch_fits(lc.lattice, lc.nc, kp.nx, kp.ny) || lc.zlen < 1 || kp.nz < 2) return hipErrorInvalidValue;
    const int tx = kp.nx / kZX, ty = kp.ny / kZY, nzc = (kp.nz + lc.zlen - 1) / lc.zlen;
    const int nb = tx * ty * nzc;
    const int ch = xcd_chunk_for(lc, nb);
    const int nt = lc.nt_store ? 1 : 0;
    const int zorder = lc.zorder;
    const dim3 grid = zorder == 1 ? dim3(zmarch_grid(tx, ty, nzc)) : grid_remapped(nb, ch);
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        if constexpr (LAT == 1 && NC == 3) {
            if (lc.csplit) {  // one component per 256-thread group
                if (lc.mrt)
                    k_collide_zmarch_iso_cs<NC, P, true><<<grid, 256 * NC, 0, lc.stream>>>(
                        kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in, (P*)fsum_out, lc.zlen, ch, nt, zorder);
                else
                    k_collide_zmarch_iso_cs<NC, P, false><<<grid, 256 * NC, 0, lc.stream>>>(
                        kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in, (P*)fsum_out, lc.zlen, ch, nt, zorder);
                return;
            }
        }
        if constexpr (LAT == 1 && NC <= 3) {
            if (lc.mrt)
                k_collide_zmarch_iso<NC, P, true><<<grid, 256, 0, lc.stream>>>(
                    kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in, (P*)fsum_out, lc.zlen, ch, nt, zorder);
            else
                k_collide_zmarch_iso<NC, P, false><<<grid, 256, 0, lc.stream>>>(
                    kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in, (P*)fsum_out, lc.zlen, ch, nt, zorder);
        }
    });
    return hipGetLastError();
}

hipError_t launch_init(const LaunchCfg& lc, const KParams& kp, const double* rho_molar, const double* u,
                       void* g, float* rref, void* fsum) {
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        k_init<LAT, NC, P><<<grid_for(kp.N, 256), 256, 0, lc.stream>>>(kp, rho_molar, u, (P*)g, rref,
                                                                        (P*)fsum);
    });
    return hipGetLastError();
}

hipError_t launch_fields(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                         const void* fsum, double* rho_molar, double* u, double* p, double* lnf) {
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        k_fields<LAT, NC, P><<<grid_for(kp.N, 256), 256, 0, lc.stream>>>(kp, (const P*)g, rref, (const P*)fsum,
                                                                          rho_molar, u, p, lnf);
    });
    return hipGetLastError();
}

hipError_t launch_export_pops(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                              double* out) {
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        k_export_pops<LAT, NC, P><<<grid_for(kp.N, 256), 256, 0, lc.stream>>>(kp, (const P*)g, rref, out);
    });
    return hipGetLastError();
}

int reduce_blocks(int N) { return (N + kRedBlock - 1) / kRedBlock; }

hipError_t launch_reduce(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref,
                         double* snap, double* partial, double* out) {
    const int nb = reduce_blocks(kp.N);
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        k_reduce_partials<LAT, NC, P><<<nb, kRedBlock, 0, lc.stream>>>(kp, (const P*)g, rref, snap, partial);
        k_reduce_final<NC><<<1, kRedBlock, 0, lc.stream>>>(partial, nb, out);
    });
    return hipGetLastError();
}


// Densities of the current populations into snap (residual baseline).
template <int LAT, int NC, typename P>
__global__ __launch_bounds__(256) void k_snapshot(KParams kp, const P* __restrict__ g, const float* __restrict__ rref,
                                                  double* __restrict__ snap) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= kp.N) return;
    P gv[NC][L::Q];
    load_pops<L, NC, P>(g, n, kp.N, gv);
    double rho[NC], mov[NC];
    densities<L, NC, P>(gv, rref, n, kp.N, rho, mov);
#pragma unroll
    for (int c = 0; c < NC; ++c) snap[(size_t)c * kp.N + n] = rho[c];
}

hipError_t launch_snapshot(const LaunchCfg& lc, const KParams& kp, const void* g, const float* rref, double* snap) {
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        k_snapshot<LAT, NC, P><<<grid_for(kp.N, 256), 256, 0, lc.stream>>>(kp, (const P*)g, rref, snap);
    });
    return hipGetLastError();
}


// ------------------------------------------------------------- fused step
// One launch per step on a D3Q19 lattice.  XCD k (hardware block b runs on
// XCD b % 8) owns the y-rows [Y0, Y1) of every plane and sweeps z.  Block j of
// the XCD computes steps 1-5 (densities and ln f) for tile t = j % tA of
// A-plane a = j / tA (a = 0 .. nz+3), where A-plane a is plane z = a - 2
// (wrapped, so planes 0 and 1 are computed again at the end of the sweep)
// restricted to the rows Y0-2 .. Y1+1 (the two halo rows on each side are
// recomputed by both neighbouring XCDs; all recomputations give identical
// values), and counts the tile in the XCD's counter of that A-plane.  It then runs steps 6-9 for tile t of plane
// z = a - 5 restricted to the rows [Y0, Y1): that needs ln f and densities of
// A-planes z .. z+4, all complete once A-plane a-1 is, which only lower-
// numbered blocks of the same XCD compute.  So every wait is on blocks
// dispatched before, the launch always drains, and the waits are bounded
// anyway.  The densities and ln f a block reads were written through its own
// XCD's L2 (rows are whole 128-byte lines, so no line is read before all of it
// is written); the second read of the populations, 5 band-planes after the
// first, comes from the Infinity Cache.
template <int LAT, int NC, typename P, bool MRT>
__global__ __launch_bounds__(256) void k_fused_step(KParams kp, const P* __restrict__ g, P* __restrict__ gn,
                                                    const float* __restrict__ rref, double* __restrict__ rt,
                                                    double* __restrict__ lnf, const P* fsum_in, P* fsum_out,
                                                    unsigned* __restrict__ counters, int* __restrict__ err,
                                                    FusedCfg fc) {
    const int k = blockIdx.x & 7;
    const int j = blockIdx.x >> 3;
    if (threadIdx.x == 0) {
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        if ((int)(xcc & 0xf) != k) atomicOr(err, kErrXcd);
    }
    const int nx = kp.nx, ny = kp.ny, nz = kp.nz;
    const int Y0 = (int)((long long)k * ny / 8);
    const int Y1 = (int)((long long)(k + 1) * ny / 8);
    const int rowsA = Y1 - Y0 + 4, rowsB = Y1 - Y0;
    const int a = j / fc.tpp;          // A-plane of this block
    const int t = j - a * fc.tpp;      // tile within the band-plane
    const int pos = t * 256 + threadIdx.x;
    unsigned* cnt = counters + (size_t)k * fc.cstride;
    // steps 1-5: tile t of A-plane a
    if (a < nz + 4) {
        if (pos < rowsA * nx) {
            const int rl = pos / nx, x = pos - rl * nx;
            int y = Y0 - 2 + rl;
            y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
            int z = a - 2;
            z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
            if (!node_moments_eos<LAT, NC, P>(kp, x + nx * (y + ny * z), kp.N, g, rref, rt, lnf))
                atomicOr(err, kErrDomain);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have reached the L2
        __syncthreads();
        if (threadIdx.x == 0) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __hip_atomic_fetch_add(&cnt[a], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // steps 6-9: tile t of plane z = a - 5, rows [Y0, Y1)
    const int zb = a - 5;
    if (zb >= 0 && zb < nz) {
        if (threadIdx.x == 0) {
            for (int q = 0; q < 5; ++q) {
                int spins = 0;
                while ((int)(__hip_atomic_load(&cnt[zb + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                             fc.target) < 0) {
                    if (++spins > fc.spin_limit) {
                        atomicOr(err, kErrWait);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        __syncthreads();
        if (pos < rowsB * nx) {
            const int rl = pos / nx, x = pos - rl * nx;
            const Dims dm{nx, ny, nz, kp.N};
            node_collide_stream<LAT, NC, P, MRT>(kp, dm, x + nx * (Y0 + rl + ny * zb), g, gn, rref, rt, lnf,
                                                 fsum_in, fsum_out, false);
        }
    }
}

hipError_t launch_fused_step(const LaunchCfg& lc, const KParams& kp, const void* g, void* gn, const float* rref,
                             double* rt, double* lnf, const void* fsum_in, void* fsum_out, unsigned* counters,
                             int* err, const FusedCfg& fc) {
    const dim3 grid(8 * (kp.nz + 5) * fc.tpp);
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        if (lc.mrt)
            k_fused_step<LAT, NC, P, true><<<grid, 256, 0, lc.stream>>>(
                kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in, (P*)fsum_out, counters, err, fc);
        else
            k_fused_step<LAT, NC, P, false><<<grid, 256, 0, lc.stream>>>(
                kp, (const P*)g, (P*)gn, rref, rt, lnf, (const P*)fsum_in, (P*)fsum_out, counters, err, fc);
    });
    return hipGetLastError();
}

// Hardware XCD of every block of a grid (to check the b % 8 placement).
__global__ void k_xcd_ids(int* out, int nblocks) {
    if (threadIdx.x == 0 && (int)blockIdx.x < nblocks) {
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        out[blockIdx.x] = (int)(xcc & 0xf);
    }
}

hipError_t launch_xcd_ids(int* out, int nblocks, hipStream_t stream) {
    k_xcd_ids<<<nblocks, 64, 0, stream>>>(out, nblocks);
    return hipGetLastError();
}

// ------------------------------------------------------------ batched server
// A request is advanced by one workgroup, or by G workgroups of one XCD that
// each own a contiguous range of its nodes.  The two phases of a step are
// separated by barriers (phase B reads the densities and ln f written in phase
// A, phase A of the next step the populations pushed in phase B): a workgroup
// barrier for G = 1, group_barrier across the G workgroups otherwise.  Every
// thread owns the same nodes in every step, and the residual check every
// check_every request steps is a max-reduction over the request.  The result
// does not depend on G, on other requests or on where the tick boundaries fall.

// Barrier across the G workgroups of one request, all on one XCD (one L2):
// each thread's stores and atomics are complete at the L2 before the workgroup
// counts in; after the count is reached, the CU's L1 is invalidated so that
// loads see the other workgroups' stores (an invalidation at workgroup scope
// leaves the L1 as it is: measured, stale neighbour values).  The wait is bounded: past the limit
// the request is flagged failed (bad bit 2) instead of waiting on.
constexpr long kGroupSpinLimit = 1L << 20;
__device__ __forceinline__ void group_barrier(GroupSync* gs, unsigned& epoch, int G) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    epoch += (unsigned)G;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        long spins = 0;
        while (__hip_atomic_load(&gs->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            if (++spins > kGroupSpinLimit) {
                __hip_atomic_fetch_or(&gs->bad, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    // device-scope acquire: invalidates this CU's L1 (the L2 is shared by the
    // group, and device memory lines stay valid there)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <int LAT, int NC, typename P, bool MRT, int kServeBlock>
__global__ __launch_bounds__(kServeBlock) void k_serve_tick(KParams kp, char* __restrict__ pool,
                                                            SlotDesc* __restrict__ descs,
                                                            const int2* __restrict__ table, GroupSync* sync,
                                                            long long steps, long long clock_budget) {
    using L = Lat<LAT>;
    __shared__ SlotDesc sd;
    __shared__ int s_bad;
    __shared__ int s_go;
    __shared__ unsigned long long s_t0;
    __shared__ double s_red[2 * NC][kServeBlock / 64];
    const int2 job = table[blockIdx.x];
    if (job.x < 0) return;  // whole workgroup, before any barrier
    if (threadIdx.x == 0) {
        sd = descs[job.x];
        s_bad = 0;
        s_t0 = wall_clock64();
    }
    __syncthreads();
    if (sd.status != kSlotRunning) return;
    const int G = sd.groups > 0 ? sd.groups : 1, m = job.y;
    GroupSync* gs = sync + job.x;
    unsigned epoch = 0;
    const Dims dm{sd.nx, sd.ny, sd.nz, sd.N};
    const size_t N = sd.N;
    // this workgroup's nodes
    const int lo = (int)((long long)sd.N * m / G), hi = (int)((long long)sd.N * (m + 1) / G);
    P* pops[2] = {(P*)(pool + sd.off_pop[0]), (P*)(pool + sd.off_pop[1])};
    double* rt = (double*)(pool + sd.off_rt);
    double* lnf = (double*)(pool + sd.off_lnf);
    P* fsum = (P*)(pool + sd.off_fsum);
    const float* rref = sizeof(P) == 4 ? (const float*)(pool + sd.off_rref) : nullptr;
    double* snap = (double*)(pool + sd.off_snap);
    int cur = sd.cur;
    long long done = sd.steps;
    int status = kSlotRunning;
    double residual = sd.residual;
    for (long long s = 0; s < steps; ++s) {
        if (done >= sd.max_steps) {
            status = kSlotMaxSteps;
            break;
        }
        if (clock_budget > 0 && (s & 7) == 0) {
            // time slice, decided every 8 steps by workgroup 0 (a slice overruns
            // its budget by at most 8 steps); every thread of the request sees
            // the same decision.  The next write of the decision is 8 steps and
            // at least 16 barriers later, so no second barrier is needed before it.
            if (G == 1) {
                if (threadIdx.x == 0) s_go = (long long)(wall_clock64() - s_t0) < clock_budget;
                __syncthreads();
            } else {
                if (m == 0 && threadIdx.x == 0)
                    __hip_atomic_store(&gs->go, (long long)(wall_clock64() - s_t0) < clock_budget ? 1 : 0,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                group_barrier(gs, epoch, G);
                if (threadIdx.x == 0) s_go = __hip_atomic_load(&gs->go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
            }
            if (!s_go) break;
        }
        bool ok = true;
        for (int n = lo + threadIdx.x; n < hi; n += kServeBlock)
            ok = node_moments_eos<LAT, NC, P>(kp, n, N, pops[cur], rref, rt, lnf) && ok;
        if (G == 1) {
            if (!ok) s_bad = 1;
            __syncthreads();
        } else {
            if (!ok) __hip_atomic_fetch_or(&gs->bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            group_barrier(gs, epoch, G);
            if (threadIdx.x == 0) s_bad = __hip_atomic_load(&gs->bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        if (s_bad) {
            status = kSlotNumeric;
            break;
        }
        for (int n = lo + threadIdx.x; n < hi; n += kServeBlock)
            node_collide_stream<LAT, NC, P, MRT>(kp, dm, n, pops[cur], pops[1 - cur], rref, rt, lnf, fsum, fsum,
                                                 false);
        if (G == 1)
            __syncthreads();
        else
            group_barrier(gs, epoch, G);
        cur = 1 - cur;
        ++done;
        if (done % sd.check_every == 0) {
            // rate residual against the snapshot of check_every steps ago
            double mdiff[NC], mrho[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) mdiff[c] = mrho[c] = 0.0;
            for (int n = lo + threadIdx.x; n < hi; n += kServeBlock) {
                P gv[NC][L::Q];
                load_pops<L, NC, P>(pops[cur], n, N, gv);
                double rho[NC], mov[NC];
                densities<L, NC, P>(gv, rref, n, N, rho, mov);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    mdiff[c] = fmax(mdiff[c], fabs(rho[c] - snap[(size_t)c * N + n]));
                    mrho[c] = fmax(mrho[c], fabs(rho[c]));
                    snap[(size_t)c * N + n] = rho[c];
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c)
                for (int off = 32; off > 0; off >>= 1) {
                    mdiff[c] = fmax(mdiff[c], __shfl_xor(mdiff[c], off));
                    mrho[c] = fmax(mrho[c], __shfl_xor(mrho[c], off));
                }
            const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
            if (lane == 0)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    s_red[c][wave] = mdiff[c];
                    s_red[NC + c][wave] = mrho[c];
                }
            __syncthreads();
            double md[NC], mr[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                md[c] = mr[c] = 0.0;
                for (int w = 0; w < kServeBlock / 64; ++w) {
                    md[c] = fmax(md[c], s_red[c][w]);
                    mr[c] = fmax(mr[c], s_red[NC + c][w]);
                }
            }
            if (G > 1) {
                // the request's maxima from every workgroup's
                if (threadIdx.x == 0)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        gs->part[m][c] = md[c];
                        gs->part[m][NC + c] = mr[c];
                    }
                group_barrier(gs, epoch, G);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    md[c] = mr[c] = 0.0;
                    for (int k = 0; k < G; ++k) {
                        md[c] = fmax(md[c], gs->part[k][c]);
                        mr[c] = fmax(mr[c], gs->part[k][NC + c]);
                    }
                }
            }
            double r = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double rc = md[c] / ((double)sd.check_every * mr[c]);
                r = (rc > r || rc != rc) ? rc : r;
            }
            residual = r;
            __syncthreads();
            if (!(r == r)) {
                status = kSlotNumeric;
                break;
            }
            if (r < sd.tol) {
                status = kSlotConverged;
                break;
            }
        }
    }
    if (status == kSlotRunning && done >= sd.max_steps) status = kSlotMaxSteps;
    if (G > 1 && status == kSlotRunning && (__hip_atomic_load(&gs->bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2))
        status = kSlotNumeric;  // a group barrier timed out
    if (m == 0 && threadIdx.x == 0) {
        descs[job.x].steps = done;
        descs[job.x].cur = cur;
        descs[job.x].residual = residual;
        descs[job.x].status = status;
    }
}

hipError_t serve_resident_blocks(const LaunchCfg& lc, int* blocks) {
    *blocks = 0;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        auto go = [&](auto bsc) {
            constexpr int BS = decltype(bsc)::value;
            e = lc.mrt ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_serve_tick<LAT, NC, P, true, BS>, BS, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_serve_tick<LAT, NC, P, false, BS>, BS, 0);
        };
        if (lc.serve_block >= 1024)
            go(std::integral_constant<int, 1024>{});
        else if (lc.serve_block >= 512)
            go(std::integral_constant<int, 512>{});
        else
            go(std::integral_constant<int, 256>{});
    });
    if (e == hipSuccess) *blocks = cus * (per_cu > 0 ? per_cu : 1);
    return e;
}

hipError_t launch_serve_tick(const LaunchCfg& lc, const KParams& kp, char* pool, SlotDesc* descs,
                             const int2* table, int nblocks, GroupSync* sync, long long steps,
                             long long clock_budget) {
    if (nblocks <= 0) return hipSuccess;
    dispatch(lc.lattice, lc.nc, lc.precision, [&](auto latc, auto ncc, auto pt) {
        FL_TYPES;
        auto go = [&](auto bsc) {
            constexpr int BS = decltype(bsc)::value;
            if (lc.mrt)
                k_serve_tick<LAT, NC, P, true, BS><<<nblocks, BS, 0, lc.stream>>>(kp, pool, descs, table, sync, steps,
                                                                                 clock_budget);
            else
                k_serve_tick<LAT, NC, P, false, BS><<<nblocks, BS, 0, lc.stream>>>(kp, pool, descs, table, sync, steps,
                                                                                  clock_budget);
        };
        if (lc.serve_block >= 1024)
            go(std::integral_constant<int, 1024>{});
        else if (lc.serve_block >= 512)
            go(std::integral_constant<int, 512>{});
        else
            go(std::integral_constant<int, 256>{});
    });
    return hipGetLastError();
}

}  // namespace fl
