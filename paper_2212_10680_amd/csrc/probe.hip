// Memory-bandwidth probe for the roofline of the benchmark (not part of the
// solver library): attainable HBM rates for the access patterns the update
// kernels use.  Each pattern reads S streams of W floats per node and writes
// them back, either to the same node (aligned) or to node (i + d_s) mod N with
// d_s the D3Q19 velocity offsets on a 128^3 lattice (the push streaming
// pattern); plus read-only streams and a plain one-stream copy.  Buffers are
// sized above the 256 MB memory-side cache.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kN = 1 << 21;  // nodes (128^3); power of two: (i + d) & (kN - 1) stays in range
constexpr int kMaxS = 40;

struct Streams {
    float* p[kMaxS];
    int d[kMaxS];
};

template <int S, int W>
__global__ __launch_bounds__(256) void k_rw(Streams in, Streams out, int shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kN) return;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = shift ? ((i + in.d[s]) & (kN - 1)) : i;
        if constexpr (W == 1) {
            out.p[s][j] = in.p[s][i] * 1.0001f;
        } else if constexpr (W == 2) {
            float2 v = reinterpret_cast<const float2*>(in.p[s])[i];
            v.x *= 1.0001f;
            v.y *= 1.0001f;
            reinterpret_cast<float2*>(out.p[s])[j] = v;
        } else {
            float4 v = reinterpret_cast<const float4*>(in.p[s])[i];
            v.x *= 1.0001f;
            v.y *= 1.0001f;
            v.z *= 1.0001f;
            v.w *= 1.0001f;
            reinterpret_cast<float4*>(out.p[s])[j] = v;
        }
    }
}

template <int S, int W>
__global__ __launch_bounds__(256) void k_read(Streams in, float* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kN) return;
    float a = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if constexpr (W == 1) {
            a += in.p[s][i];
        } else {
            const float2 v = reinterpret_cast<const float2*>(in.p[s])[i];
            a += v.x + v.y;
        }
    }
    out[i] = a;
}

__global__ void k_copy(const float4* a, float4* b, long n4) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) b[i] = a[i];
}

// ---- visiting orders of the three-component collide pass (256^3 lattice,
// 57 population streams of 4 B in and out, push-shifted destinations, no
// arithmetic and no stencil fields): one thread per node in node order, or
// z-marching workgroups of 256 threads that own a tile of the (x, y) plane and
// march 16 planes, taken in XCD-contiguous chunks or in XCD y-bands (all XCDs
// in the same planes).  LDS padding holds one workgroup per CU, as in the
// collide kernel.  Each thread loads all its streams before it stores.
constexpr int kMX = 256, kMY = 256, kMZ = 256;
constexpr int kMN = kMX * kMY * kMZ;
constexpr int kMS = 57;
struct MStreams {
    float* p[kMS];
};
__constant__ int c_ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int c_ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int c_ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__device__ __forceinline__ int mlin(int x, int y, int z) { return x + kMX * (y + kMY * z); }

// ORDER 0: node order, one node per thread; 1: z-march, XCD-contiguous chunks;
// 2: z-march, XCD y-bands.  TW: tile width (tile height 256 / TW).  XSHIFT:
// destinations shifted along x too (false: y and z only).
template <int ORDER, int TW, bool XSHIFT>
__global__ __launch_bounds__(256) void k_zorder(MStreams in, MStreams out) {
    __shared__ float pad[24 * 1024];  // 96 KB: one workgroup per CU
    if (threadIdx.x == 1023) pad[blockIdx.x & 1023] = 0.f;  // never taken: keeps the array
    const int t = threadIdx.x;
    auto node = [&](int x, int y, int z) {
        float v[kMS];
        const int n = mlin(x, y, z);
#pragma unroll
        for (int s = 0; s < kMS; ++s) v[s] = __builtin_nontemporal_load(&in.p[s][n]);
#pragma unroll
        for (int s = 0; s < kMS; ++s) {
            const int a = s % 19;
            const int xx = XSHIFT ? (x + c_ex[a]) & (kMX - 1) : x;
            out.p[s][mlin(xx, (y + c_ey[a]) & (kMY - 1), (z + c_ez[a]) & (kMZ - 1))] = v[s] * 1.0001f;
        }
    };
    if (ORDER == 0) {
        const int n = blockIdx.x * 256 + t;
        node(n & (kMX - 1), (n / kMX) & (kMY - 1), n / (kMX * kMY));
        return;
    }
    constexpr int TH = 256 / TW, TX = kMX / TW, TY = kMY / TH, ZL = 16;
    constexpr int tiles = TX * TY, nb = tiles * (kMZ / ZL);
    const int b = blockIdx.x;
    int zc, txy;
    if (ORDER == 1) {
        const int lb = (b & 7) * (nb / 8) + (b >> 3);
        zc = lb / tiles;
        txy = lb % tiles;
    } else {
        const int k = b & 7, j = b >> 3, per = tiles / 8;
        zc = j / per;
        const int tl = j % per;
        txy = (k * (per / TX) + tl / TX) * TX + tl % TX;
    }
    const int x = (txy % TX) * TW + t % TW, y = (txy / TX) * TH + t / TW;
    for (int z = zc * ZL; z < zc * ZL + ZL; ++z) node(x, y, z);
}

}  // namespace

extern "C" {

// Runs each visiting order of k_zorder (10 launches, HIP events) and writes
// one line per order into `report` (at most `cap` bytes, NUL-terminated).
// Returns 0, or -1 on a HIP error (the report names it).  Allocates 7.7 GB.
int flp_zmarch_probe(char* report, int cap) {
    int used = 0;
    auto put = [&](const char* fmt, auto... a) {
        if (used < cap) used += snprintf(report + used, (size_t)(cap - used), fmt, a...);
    };
    MStreams in{}, out{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    auto ck = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == 0) {
            put("HIP error %s in %s\n", hipGetErrorString(e), what);
            rc = -1;
        }
        return rc == 0;
    };
    for (int s = 0; s < kMS && rc == 0; ++s) {
        ck(hipMalloc(&in.p[s], (size_t)kMN * 4), "hipMalloc");
        if (rc == 0) ck(hipMalloc(&out.p[s], (size_t)kMN * 4), "hipMalloc");
        if (rc == 0) ck(hipMemset(in.p[s], 0, (size_t)kMN * 4), "hipMemset");
    }
    if (rc == 0) ck(hipEventCreate(&e0), "hipEventCreate");
    if (rc == 0) ck(hipEventCreate(&e1), "hipEventCreate");
    auto run = [&](const char* name, auto launch) {
        if (rc) return;
        launch();
        if (!ck(hipDeviceSynchronize(), name)) return;
        ck(hipEventRecord(e0), name);
        for (int r = 0; r < 10; ++r) launch();
        ck(hipEventRecord(e1), name);
        if (!ck(hipEventSynchronize(e1), name)) return;
        float ms = 0.f;
        ck(hipEventElapsedTime(&ms, e0, e1), name);
        ms /= 10.f;
        const double bytes = 2.0 * kMS * 4.0 * kMN;
        put("%-58s %8.3f ms %6.0f GB/s\n", name, ms, bytes / (ms * 1e-3) / 1e9);
    };
    const int nz = (kMX / 64) * (kMY / 4) * (kMZ / 16);
    run("57 x 4 B push-shifted, node order", [&] { k_zorder<0, 64, true><<<kMN / 256, 256>>>(in, out); });
    run("57 x 4 B push-shifted, z-march 64x4, XCD chunks", [&] { k_zorder<1, 64, true><<<nz, 256>>>(in, out); });
    run("57 x 4 B push-shifted, z-march 64x4, XCD y-bands", [&] { k_zorder<2, 64, true><<<nz, 256>>>(in, out); });
    run("57 x 4 B shifted in y, z only, z-march 64x4, XCD y-bands",
        [&] { k_zorder<2, 64, false><<<nz, 256>>>(in, out); });
    run("57 x 4 B push-shifted, z-march 128x2, XCD y-bands", [&] { k_zorder<2, 128, true><<<nz, 256>>>(in, out); });
    run("57 x 4 B push-shifted, z-march 256x1 (whole rows), XCD y-bands",
        [&] { k_zorder<2, 256, true><<<nz, 256>>>(in, out); });
    for (int s = 0; s < kMS; ++s) {
        if (in.p[s]) (void)hipFree(in.p[s]);
        if (out.p[s]) (void)hipFree(out.p[s]);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}


// Runs every pattern (10 launches each, HIP events) and writes one line per
// pattern into `report` (at most `cap` bytes, NUL-terminated).  Returns 0, or
// -1 on a HIP error (the report then names it).  Allocates about 3.8 GB.
int flp_stream_probe(char* report, int cap) {
    int used = 0;
    auto put = [&](const char* fmt, auto... a) {
        if (used < cap) used += snprintf(report + used, (size_t)(cap - used), fmt, a...);
    };
    Streams in{}, out{};
    float* sink = nullptr;
    float *A = nullptr, *B = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    const int dirs[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                             {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                             {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                             {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    const long n4 = 38L * kN / 4;  // one 608 MB copy
    auto ck = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == 0) {
            put("HIP error %s in %s\n", hipGetErrorString(e), what);
            rc = -1;
        }
        return rc == 0;
    };
    for (int s = 0; s < kMaxS && rc == 0; ++s) {
        ck(hipMalloc(&in.p[s], (size_t)kN * 16), "hipMalloc");
        if (rc == 0) ck(hipMalloc(&out.p[s], (size_t)kN * 16), "hipMalloc");
        if (rc == 0) ck(hipMemset(in.p[s], 0, (size_t)kN * 16), "hipMemset");
        const int* e = dirs[s % 19];
        in.d[s] = out.d[s] = e[0] + 128 * e[1] + 128 * 128 * e[2];
    }
    if (rc == 0) ck(hipMalloc(&sink, (size_t)kN * 4), "hipMalloc");
    if (rc == 0) ck(hipMalloc(&A, (size_t)n4 * 16), "hipMalloc");
    if (rc == 0) ck(hipMalloc(&B, (size_t)n4 * 16), "hipMalloc");
    if (rc == 0) ck(hipMemset(A, 0, (size_t)n4 * 16), "hipMemset");
    if (rc == 0) ck(hipEventCreate(&e0), "hipEventCreate");
    if (rc == 0) ck(hipEventCreate(&e1), "hipEventCreate");
    auto run = [&](const char* name, double bytes, auto launch) {
        if (rc) return;
        launch();
        if (!ck(hipDeviceSynchronize(), name)) return;
        ck(hipEventRecord(e0), name);
        for (int r = 0; r < 10; ++r) launch();
        ck(hipEventRecord(e1), name);
        if (!ck(hipEventSynchronize(e1), name)) return;
        float ms = 0.f;
        ck(hipEventElapsedTime(&ms, e0, e1), name);
        ms /= 10.f;
        put("%-44s %9.1f us %8.0f GB/s\n", name, ms * 1e3, bytes / (ms * 1e-3) / 1e9);
    };
    const int g = kN / 256;
    const double node = (double)kN;
    run("read 38 x 4 B streams", 38.0 * 4 * node + 4 * node, [&] { k_read<38, 1><<<g, 256>>>(in, sink); });
    run("read 19 x 8 B streams", 19.0 * 8 * node + 4 * node, [&] { k_read<19, 2><<<g, 256>>>(in, sink); });
    for (int sh = 0; sh < 2; ++sh) {
        const char* t = sh ? "push-shifted" : "aligned";
        char nm[64];
        snprintf(nm, sizeof nm, "in+out 38 x 4 B, %s", t);
        run(nm, 2.0 * 38 * 4 * node, [&] { k_rw<38, 1><<<g, 256>>>(in, out, sh); });
        snprintf(nm, sizeof nm, "in+out 19 x 8 B, %s", t);
        run(nm, 2.0 * 19 * 8 * node, [&] { k_rw<19, 2><<<g, 256>>>(in, out, sh); });
        snprintf(nm, sizeof nm, "in+out 10 x 16 B, %s", t);
        run(nm, 2.0 * 10 * 16 * node, [&] { k_rw<10, 4><<<g, 256>>>(in, out, sh); });
    }
    run("copy, one 608 MB stream", 2.0 * n4 * 16,
        [&] { k_copy<<<(unsigned)((n4 + 255) / 256), 256>>>((const float4*)A, (float4*)B, n4); });
    for (int s = 0; s < kMaxS; ++s) {
        if (in.p[s]) (void)hipFree(in.p[s]);
        if (out.p[s]) (void)hipFree(out.p[s]);
    }
    if (sink) (void)hipFree(sink);
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
