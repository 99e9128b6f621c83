// Memory-pattern probes: the HBM streams of the mixed-precision D3Q19 + D3Q7
// step (19 fp16 g populations and 6 fp32 h populations per node, each read
// once and written once, plane-major [z][q][plane]) with no arithmetic, in
// the step kernel's launch shape. They measure the ceiling the step kernel
// can reach with its access pattern:
//   PFLBM_PROBE_CHUNKS    contiguous 1024-node chunks of each population plane
//   PFLBM_PROBE_TILES     256 x 4 tiles, workgroups in XCD runs, z blocks
//                         marched, aligned loads and stores (the step's pull
//                         without shifts)
//   PFLBM_PROBE_SHIFT_LD  PFLBM_PROBE_TILES with the loads of the ten g
//                         populations with c_x != 0 taken from x - c_x (the
//                         pull of the step kernel)
//   PFLBM_PROBE_SHIFT_ST  PFLBM_PROBE_TILES with those populations stored at
//                         x + c_x (the in-place schemes' shifted stores)
//   PFLBM_PROBE_ZSKEW     PFLBM_PROBE_SHIFT_LD with, when one z block spans
//                         the box, each workgroup starting its march at its
//                         own plane (spread evenly over nz) and wrapping
// Loads are ordinary and stores non-temporal, as in the step kernel.
// Every index is wrapped into the box, so the probes stay inside the buffers
// for any box.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.h"
#include "pflbm.h"

namespace pfk {
namespace {

constexpr int PQG = 19, PQH = 6;
constexpr int PTX = 256, PTY = 4, PNT = PTX * PTY;

struct ProbeArgs {
    const uint16_t* gs;
    uint16_t* gd;
    const float* hs;
    float* hd;
    int nx, ny, nz, P, zb, ntx, nty;
};

__device__ __forceinline__ int remap_xcd(int bid, int nb) {
    const int per = nb / 8;
    if (bid >= per * 8) return bid;
    return (bid % 8) * per + bid / 8;
}

template <int PATTERN>
__global__ __launch_bounds__(PNT) void k_probe(const ProbeArgs a) {
    int x, y, zs;
    bool active;
    if constexpr (PATTERN == PFLBM_PROBE_CHUNKS) {
        const int nch = (a.P + PNT - 1) / PNT;
        const int b = blockIdx.x;
        const int ch = b % nch, bz = b / nch;
        const int n = ch * PNT + threadIdx.x;
        active = n < a.nx * a.ny;
        y = active ? n / a.nx : 0;
        x = active ? n - y * a.nx : 0;
        zs = bz * a.zb;
    } else {
        const int b = remap_xcd(blockIdx.x, gridDim.x);
        const int bx = b % a.ntx, byz = b / a.ntx;
        const int by = byz % a.nty, bz = byz / a.nty;
        x = bx * PTX + (int)threadIdx.x % PTX;
        y = by * PTY + (int)threadIdx.x / PTX;
        active = x < a.nx && y < a.ny;
        zs = bz * a.zb;
    }
    if (!active) return;
    int ze = min(a.nz, zs + a.zb);
    if constexpr (PATTERN == PFLBM_PROBE_ZSKEW) {
        if (a.zb >= a.nz) {
            const int nb = gridDim.x, b = remap_xcd(blockIdx.x, gridDim.x);
            zs = (int)(((long long)b * a.nz) / nb);
            ze = zs + a.nz;
        }
    }
    const int own = y * a.nx + x;
    for (int zv = zs; zv < ze; ++zv) {
        const int z = zv < a.nz ? zv : zv - a.nz;
        const size_t gb = (size_t)z * PQG * a.P, hb = (size_t)z * PQH * a.P;
        uint16_t gv[PQG];
        unroll<PQG>([&](auto I) {
            constexpr int i = I;
            constexpr int cx = D3Q19::c(i, 0);
            int src = own;
            if constexpr ((PATTERN == PFLBM_PROBE_SHIFT_LD || PATTERN == PFLBM_PROBE_ZSKEW) && cx != 0) {
                int xs = x - cx;
                xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
                src = y * a.nx + xs;
            }
            gv[i] = a.gs[gb + (size_t)i * a.P + src];
        });
        float hv[PQH];
        unroll<PQH>([&](auto J) {
            constexpr int q = J;
            hv[q] = a.hs[hb + (size_t)q * a.P + own];
        });
        unroll<PQG>([&](auto I) {
            constexpr int i = I;
            constexpr int cx = D3Q19::c(i, 0);
            int dst = own;
            if constexpr (PATTERN == PFLBM_PROBE_SHIFT_ST && cx != 0) {
                int xd = x + cx;
                xd = xd < 0 ? xd + a.nx : (xd >= a.nx ? xd - a.nx : xd);
                dst = y * a.nx + xd;
            }
            __builtin_nontemporal_store(gv[i], &a.gd[gb + (size_t)i * a.P + dst]);
        });
        unroll<PQH>([&](auto J) {
            constexpr int q = J;
            __builtin_nontemporal_store(hv[q], &a.hd[hb + (size_t)q * a.P + own]);
        });
    }
}

size_t probe_plane(int nx, int ny) { return ((size_t)nx * ny + 63) / 64 * 64; }

}  // namespace
}  // namespace pfk

using namespace pfk;

extern "C" {

int pflbm_probe_bytes(int nx, int ny, int nz, size_t* g_bytes, size_t* h_bytes) {
    if (nx < 1 || ny < 1 || nz < 1 || !g_bytes || !h_bytes) return PFLBM_EINVAL;
    if ((long long)nx * ny * nz > 0x7fffffffLL) return PFLBM_EINVAL;
    const size_t P = probe_plane(nx, ny);
    *g_bytes = (size_t)nz * PQG * P * sizeof(uint16_t);
    *h_bytes = (size_t)nz * PQH * P * sizeof(float);
    return PFLBM_OK;
}

int pflbm_probe_stream(const void* g_src, void* g_dst, const void* h_src, void* h_dst, int nx, int ny,
                       int nz, int pattern, int zblock, void* hip_stream) {
    if (!g_src || !g_dst || !h_src || !h_dst) return PFLBM_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1 || zblock < 1) return PFLBM_EINVAL;
    if ((long long)nx * ny * nz > 0x7fffffffLL) return PFLBM_EINVAL;
    if (pattern < PFLBM_PROBE_CHUNKS || pattern > PFLBM_PROBE_ZSKEW) return PFLBM_EINVAL;
    ProbeArgs a;
    a.gs = (const uint16_t*)g_src;
    a.gd = (uint16_t*)g_dst;
    a.hs = (const float*)h_src;
    a.hd = (float*)h_dst;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.P = (int)probe_plane(nx, ny);
    a.zb = zblock > nz ? nz : zblock;
    a.ntx = (nx + PTX - 1) / PTX;
    a.nty = (ny + PTY - 1) / PTY;
    const int nzb = (nz + a.zb - 1) / a.zb;
    hipStream_t st = (hipStream_t)hip_stream;
    if (pattern == PFLBM_PROBE_CHUNKS) {
        const int nch = (a.P + PNT - 1) / PNT;
        hipLaunchKernelGGL(k_probe<PFLBM_PROBE_CHUNKS>, dim3(nch * nzb), dim3(PNT), 0, st, a);
    } else {
        const dim3 grid(a.ntx * a.nty * nzb);
        if (pattern == PFLBM_PROBE_TILES) hipLaunchKernelGGL(k_probe<PFLBM_PROBE_TILES>, grid, dim3(PNT), 0, st, a);
        else if (pattern == PFLBM_PROBE_SHIFT_LD) hipLaunchKernelGGL(k_probe<PFLBM_PROBE_SHIFT_LD>, grid, dim3(PNT), 0, st, a);
        else if (pattern == PFLBM_PROBE_SHIFT_ST) hipLaunchKernelGGL(k_probe<PFLBM_PROBE_SHIFT_ST>, grid, dim3(PNT), 0, st, a);
        else hipLaunchKernelGGL(k_probe<PFLBM_PROBE_ZSKEW>, grid, dim3(PNT), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? PFLBM_OK : PFLBM_EHIP;
}

}  // extern "C"
