// HIP kernels around the fused step (gfx950): initialisation, canonical
// float64 I/O, the float64 reductions (diagnostics, nonlocal multiplier) and
// the dispatch of the step kernel to its per-pair, per-model instantiations
// (step_inst.hip). The device code of the step itself is in step.h.
#include "step.h"

namespace pfk {

hipError_t launch_step(int lattice, int model, int precision, int mode, const KArgs& a, hipStream_t s) {
    using StepFn = hipError_t (*)(int, int, const KArgs&, hipStream_t);
    static const StepFn fn[3][5] = {
        {launch_step_p0_m0, launch_step_p0_m1, launch_step_p0_m2, launch_step_p0_m3, launch_step_p0_m4},
        {launch_step_p1_m0, launch_step_p1_m1, launch_step_p1_m2, launch_step_p1_m3, launch_step_p1_m4},
        {launch_step_p2_m0, launch_step_p2_m1, launch_step_p2_m2, launch_step_p2_m3, launch_step_p2_m4}};
    return fn[lattice][model](precision, mode, a, s);
}

int occupancy_step(int lattice, int model, int precision, int tile, int walls) {
    using OccFn = int (*)(int, int, int);
    static const OccFn fn[3][5] = {
        {occupancy_step_p0_m0, occupancy_step_p0_m1, occupancy_step_p0_m2, occupancy_step_p0_m3, occupancy_step_p0_m4},
        {occupancy_step_p1_m0, occupancy_step_p1_m1, occupancy_step_p1_m2, occupancy_step_p1_m3, occupancy_step_p1_m4},
        {occupancy_step_p2_m0, occupancy_step_p2_m1, occupancy_step_p2_m2, occupancy_step_p2_m3, occupancy_step_p2_m4}};
    return fn[lattice][model](precision, tile, walls);
}

// final reduction over the per-block partials, one workgroup, fixed order
__global__ __launch_bounds__(BLOCK) void k_reduce(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out) {
    DiagAcc d;
    diag_init(d);
    for (int b = threadIdx.x; b < nb; b += BLOCK) diag_combine(d.v, part + (size_t)b * NDIAG);
    block_reduce_diag(d, out);
}

__global__ void k_header(long long* dst, CkHeader hd) {
    if (threadIdx.x < CkHeader::N) dst[threadIdx.x] = hd.v[threadIdx.x];
}

// ----------------------------------------------------------------------------
// canonical (post-streaming) populations <-> stored (post-collision) buffers

// Stored element that the pull of population i at node (x, y, z) reads: slot i
// of node x - c_i, or, if that node lies beyond a wall, slot opp(i) of the node
// itself (the pull then adds the wall term of opp(i)). The map is a bijection
// of the stored elements, so canonical -> stored is its inverse scatter.
template <class L, int i, int QS, int OFF>
__device__ __forceinline__ size_t pull_source(int nx, int ny, int nz, const int* bc, int x, int y, int z, int P,
                                              bool& wall, int& side) {
    int nb;
    wall = shifted<L, i, -1>(nx, ny, nz, bc, x, y, z, nb, side);
    if (wall) return el<QS>(z, L::opp(i) - OFF, y * nx + x, P);
    const int plane = nx * ny;
    return el<QS>(nb / plane, i - OFF, nb % plane, P);
}

// ----------------------------------------------------------------------------
// initialisation: h = h_eq(phi0, u0), g = g_eq(p0 / (rho0 c_s^2), u0), written
// where the first step's pull reads them

template <class PAIR, int MODEL, int PREC>
__global__ __launch_bounds__(256) void k_init(const InitArgs a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    using T = typename Types<PREC>::T;
    using GS = typename Types<PREC>::GS;
    using HS = typename Types<PREC>::HS;
    using GC = GCodec<PREC>;
    constexpr bool D3 = PAIR::dim == 3;
    constexpr int HOFF = rest_offset(MODEL, D3);
    constexpr int QHS = HL::Q - HOFF;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int x = (int)(n % a.nx), y = (int)((n / a.nx) % a.ny), z = (int)(n / ((long long)a.nx * a.ny));
    const int ip = y * a.nx + x;
    const Phys& ph = a.ph;
    const double phi = a.phi0[n];
    double u[3] = {0.0, 0.0, 0.0};
    if (a.u0) {
        u[0] = a.u0[n];
        u[1] = a.u0[nn + n];
        if (D3) u[2] = a.u0[2 * nn + n];
    }
    const double rho = ph.rhoL + phi * ph.dRho;
    const double ps = a.p0 ? 3.0 * a.p0[n] / rho : 0.0;
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    GS* G = (GS*)a.g;
    HS* H = (HS*)a.h;
    unroll<GL::Q>([&](auto I) {
        constexpr int i = I;
        const double cu = GL::c(i, 0) * u[0] + GL::c(i, 1) * u[1] + GL::c(i, 2) * u[2];
        double geq;
        if constexpr (MODEL == 3 || MODEL == 4) {
            // Eqs. liang_feq / liang2_feq: (p/c_s^2)(w - [i = 0]) + rho w (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
            const double p0 = a.p0 ? a.p0[n] : 0.0;
            geq = 3.0 * p0 * (GL::w(i) - (i == 0 ? 1.0 : 0.0)) +
                  rho * GL::w(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        } else {
            geq = GL::w(i) * (ps + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        }
        bool w;
        int side;
        const size_t e = pull_source<GL, i, GL::Q, 0>(a.nx, a.ny, a.nz, a.bc, x, y, z, a.P, w, side);
        if (w) geq -= a.gcorr[side][GL::opp(i)];
        G[e] = GC::template enc<GL, i, GS, T>((T)geq);
    });
    auto put_h = [&](auto J, double v) {
        constexpr int al = J;
        bool w;
        int side;
        H[pull_source<HL, al, QHS, HOFF>(a.nx, a.ny, a.nz, a.bc, x, y, z, a.P, w, side)] = (HS)v;
    };
    if constexpr (MODEL == 0) {
        unroll<QHS>([&](auto J) {
            constexpr int al = J + HOFF;
            const double eu = HL::c(al, 0) * u[0] + HL::c(al, 1) * u[1] + HL::c(al, 2) * u[2];
            const double heq = HL::w(al) * phi * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
            put_h(std::integral_constant<int, al>{}, heq);
        });
    } else if constexpr (MODEL == 2 || MODEL == 3) {
        unroll<QHS>([&](auto J) {
            constexpr int al = J + HOFF;
            const double eu = HL::c(al, 0) * u[0] + HL::c(al, 1) * u[1] + HL::c(al, 2) * u[2];
            put_h(std::integral_constant<int, al>{}, HL::w(al) * phi * (1.0 + 3.0 * eu));
        });
        if constexpr (MODEL == 3) {
            T* PU = (T*)a.phiu;
            for (int c = 0; c < 3; ++c) PU[el<3>(z, c, ip, a.P)] = (T)(phi * u[c]);
        }
    } else {
        // mu_phi(phi0) with the same stencil and ghost rules as the step
        double lap = 0.0;
        unroll<GL::Q>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                const int gx = ghost_coord(x + GL::c(i, 0), a.nx, a.bc[0]);
                const int gy = ghost_coord(y + GL::c(i, 1), a.ny, a.bc[1]);
                const int gz = ghost_coord(z + GL::c(i, 2), a.nz, a.bc[2]);
                lap += 6.0 * GL::w(i) * (a.phi0[((long long)gz * a.ny + gy) * a.nx + gx] - phi);
            }
        });
        const double mu = ph.beta4 * phi * (phi - 1.0) * (phi - 0.5) - ph.kappa * lap;
        unroll<HL::Q>([&](auto J) {
            constexpr int al = J;
            double heq;
            if constexpr (al == 0) {
                heq = phi + (HL::w(0) - 1.0) * ph.eta * mu;
            } else {
                const double ep = HL::c(al, 0) * phi * u[0] + HL::c(al, 1) * phi * u[1] +
                                  HL::c(al, 2) * phi * u[2];
                heq = HL::w(al) * ph.eta * mu + 3.0 * HL::w(al) * ep;
            }
            put_h(std::integral_constant<int, al>{}, heq);
        });
        T* PU = (T*)a.phiu;
        for (int c = 0; c < 3; ++c) PU[el<3>(z, c, ip, a.P)] = (T)(phi * u[c]);
    }
}

// ----------------------------------------------------------------------------
// canonical float64 I/O

template <class PAIR, int MODEL, int PREC>
__global__ __launch_bounds__(256) void k_get(const IOArgs a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    using T = typename Types<PREC>::T;
    using GS = typename Types<PREC>::GS;
    using HS = typename Types<PREC>::HS;
    using GC = GCodec<PREC>;
    constexpr bool D3 = PAIR::dim == 3;
    constexpr int HOFF = rest_offset(MODEL, D3);
    constexpr int QHS = HL::Q - HOFF;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int x = (int)(n % a.nx), y = (int)((n / a.nx) % a.ny), z = (int)(n / ((long long)a.nx * a.ny));
    const int ip = y * a.nx + x;
    const GS* G = (const GS*)a.g;
    const HS* H = (const HS*)a.h;
    unroll<GL::Q>([&](auto I) {
        constexpr int i = I;
        bool w;
        int side;
        const size_t e = pull_source<GL, i, GL::Q, 0>(a.nx, a.ny, a.nz, a.bc, x, y, z, a.P, w, side);
        T v = GC::template dec<GL, i, GS, T>(G[e]);
        if (w) v += (T)a.gcorr[side][GL::opp(i)];
        if (a.cgf) a.cgf[(size_t)i * nn + n] = (float)v;
        else a.cg[(size_t)i * nn + n] = (double)v;
    });
    unroll<HL::Q>([&](auto J) {
        constexpr int al = J;
        double v = 0.0;
        if constexpr (al >= HOFF) {
            bool w;
            int side;
            v = (double)H[pull_source<HL, al, QHS, HOFF>(a.nx, a.ny, a.nz, a.bc, x, y, z, a.P, w, side)];
        }
        if (a.chf) a.chf[(size_t)al * nn + n] = (float)v;
        else a.ch[(size_t)al * nn + n] = v;
    });
}

template <class PAIR, int MODEL, int PREC>
__global__ __launch_bounds__(256) void k_set(const IOArgs a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    using T = typename Types<PREC>::T;
    using GS = typename Types<PREC>::GS;
    using HS = typename Types<PREC>::HS;
    using GC = GCodec<PREC>;
    constexpr bool D3 = PAIR::dim == 3;
    constexpr int HOFF = rest_offset(MODEL, D3);
    constexpr int QHS = HL::Q - HOFF;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int x = (int)(n % a.nx), y = (int)((n / a.nx) % a.ny), z = (int)(n / ((long long)a.nx * a.ny));
    const int ip = y * a.nx + x;
    GS* G = (GS*)a.g;
    HS* H = (HS*)a.h;
    unroll<GL::Q>([&](auto I) {
        constexpr int i = I;
        bool w;
        int side;
        const size_t e = pull_source<GL, i, GL::Q, 0>(a.nx, a.ny, a.nz, a.bc, x, y, z, a.P, w, side);
        double v = a.cg[(size_t)i * nn + n];
        if (w) v -= a.gcorr[side][GL::opp(i)];
        G[e] = GC::template enc<GL, i, GS, T>((T)v);
    });
    unroll<QHS>([&](auto J) {
        constexpr int al = J + HOFF;
        bool w;
        int side;
        H[pull_source<HL, al, QHS, HOFF>(a.nx, a.ny, a.nz, a.bc, x, y, z, a.P, w, side)] =
            (HS)a.ch[(size_t)al * nn + n];
    });
}

// (phi u) of the previous step, native [z][3][P] of the compute type, to or
// from canonical float64 [3][z][y][x]
template <class T, bool GET>
__global__ __launch_bounds__(256) void k_phiu_io(T* pu, double* c, int P, int nx, int ny, int nz) {
    const long long nn = (long long)nx * ny * nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int pl = nx * ny;
    const int z = (int)(n / pl), ip = (int)(n - (long long)z * pl);
    for (int k = 0; k < 3; ++k) {
        const size_t e = ((size_t)z * 3 + k) * (size_t)P + ip;
        if constexpr (GET) c[(size_t)k * nn + n] = (double)pu[e];
        else pu[e] = (T)c[(size_t)k * nn + n];
    }
}

// ----------------------------------------------------------------------------
// nonlocal multiplier: gamma = sum (4 beta/kappa)(phi* - 1) phi* (phi* - 1/2)
// / sum (1 - phi*) phi* over all nodes (Eq. lagrange_multiplier), phi* the
// post-streaming sum of h pulled from the current buffer; float64 sums in a
// fixed order (bit-reproducible)

template <class PAIR, int PREC, int WALLS>
__global__ __launch_bounds__(256) void k_gamma_part(const GammaArgs a) {
    using HL = typename PAIR::H;
    using T = typename Types<PREC>::T;
    using HS = typename Types<PREC>::HS;
    constexpr int HOFF = PAIR::dim == 3 ? 1 : 0;
    constexpr int QHS = HL::Q - HOFF;
    __shared__ double red[2][256 / 64];
    // workgroup (bx, bz): 256 consecutive in-plane nodes over GAMMA_ZB planes;
    // phi* pulled by the step's own helper in the step's summation order
    const int ip = blockIdx.x * 256 + threadIdx.x;
    const int z0 = blockIdx.y * GAMMA_ZB, z1 = min(a.nz, z0 + GAMMA_ZB);
    double num = 0.0, den = 0.0;
    if (ip < a.nx * a.ny) {
        const int x = ip % a.nx, y = ip / a.nx;
        const HS* __restrict__ H = (const HS*)a.h;
        Cross X = make_cross(x, y, a.nx, a.ny, a.bc);
        for (int zl = z0; zl < z1; ++zl) {
            const int z = __builtin_amdgcn_readfirstlane(zl);
            lane_opaque(X);
            const ZPlanes zp = make_zplanes(z, a.nz, a.bc[2]);
            T s = (T)0;
            unroll<QHS>([&](auto J) {
                constexpr int al = J + HOFF;
                s += pull_h<HL, al, HOFF, WALLS, T>(H, X, zp, a.P);
            });
            const double phi = (double)s;
            num += a.w32 * (phi - 1.0) * phi * (phi - 0.5);
            den += (1.0 - phi) * phi;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        num += __shfl_xor(num, off, 64);
        den += __shfl_xor(den, off, 64);
    }
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    if (lane == 0) {
        red[0][wv] = num;
        red[1][wv] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sn = red[0][0], sd = red[1][0];
        for (int k = 1; k < 256 / 64; ++k) {
            sn += red[0][k];
            sd += red[1][k];
        }
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.partials[2 * b] = sn;
        a.partials[2 * b + 1] = sd;
    }
}

// one workgroup of GAMMA_FINAL_THREADS, fixed summation order (bit-reproducible)
constexpr int GAMMA_FINAL_THREADS = 1024;
__global__ __launch_bounds__(GAMMA_FINAL_THREADS) void k_gamma_final(const double* __restrict__ part, long long nb,
                                                                     double* __restrict__ gamma) {
    __shared__ double red[2][GAMMA_FINAL_THREADS / 64];
    double num = 0.0, den = 0.0;
    for (long long b = threadIdx.x; b < nb; b += GAMMA_FINAL_THREADS) {
        num += part[2 * b];
        den += part[2 * b + 1];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        num += __shfl_xor(num, off, 64);
        den += __shfl_xor(den, off, 64);
    }
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    if (lane == 0) {
        red[0][wv] = num;
        red[1][wv] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sn = red[0][0], sd = red[1][0];
        for (int k = 1; k < GAMMA_FINAL_THREADS / 64; ++k) {
            sn += red[0][k];
            sd += red[1][k];
        }
        gamma[0] = sd != 0.0 ? sn / sd : 0.0;
    }
}

// ----------------------------------------------------------------------------
// dispatch

#define PFLBM_NODE_DISPATCH(KERNEL, ARGS, NN)                                               \
    do {                                                                                     \
        const dim3 grid((unsigned)(((NN) + 255) / 256)), block(256);                          \
        auto go = [&](auto pair, auto md, auto pr) {                                         \
            using P_ = decltype(pair);                                                       \
            constexpr int M_ = decltype(md)::value, R_ = decltype(pr)::value;                \
            hipLaunchKernelGGL((KERNEL<P_, M_, R_>), grid, block, 0, s, ARGS);               \
        };                                                                                   \
        auto prec = [&](auto pair, auto md) {                                                \
            switch (precision) {                                                             \
                case 0: go(pair, md, std::integral_constant<int, 0>{}); break;              \
                case 1: go(pair, md, std::integral_constant<int, 1>{}); break;              \
                case 2: go(pair, md, std::integral_constant<int, 2>{}); break;              \
                default: go(pair, md, std::integral_constant<int, 3>{});                    \
            }                                                                                \
        };                                                                                   \
        auto mdl = [&](auto pair) {                                                          \
            if (model == 4) prec(pair, std::integral_constant<int, 4>{});                    \
            else if (model == 3) prec(pair, std::integral_constant<int, 3>{});               \
            else if (model == 2) prec(pair, std::integral_constant<int, 2>{});               \
            else if (model == 1) prec(pair, std::integral_constant<int, 1>{});               \
            else prec(pair, std::integral_constant<int, 0>{});                               \
        };                                                                                   \
        if (lattice == 0) mdl(Pair2D{});                                                     \
        else if (lattice == 1) mdl(Pair3D{});                                                \
        else mdl(Pair3D27{});                                                                \
    } while (0)

hipError_t launch_init(int lattice, int model, int precision, const InitArgs& a, hipStream_t s) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    PFLBM_NODE_DISPATCH(k_init, a, nn);
    return hipGetLastError();
}

hipError_t launch_get(int lattice, int model, int precision, const IOArgs& a, hipStream_t s) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    PFLBM_NODE_DISPATCH(k_get, a, nn);
    return hipGetLastError();
}

hipError_t launch_set(int lattice, int model, int precision, const IOArgs& a, hipStream_t s) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    PFLBM_NODE_DISPATCH(k_set, a, nn);
    return hipGetLastError();
}

hipError_t launch_phiu_io(int precision, bool get, void* pu, double* canon, int P, int nx, int ny, int nz,
                          hipStream_t s) {
    const long long nn = (long long)nx * ny * nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    if (precision == 0) {
        if (get) hipLaunchKernelGGL((k_phiu_io<double, true>), grid, block, 0, s, (double*)pu, canon, P, nx, ny, nz);
        else hipLaunchKernelGGL((k_phiu_io<double, false>), grid, block, 0, s, (double*)pu, canon, P, nx, ny, nz);
    } else {
        if (get) hipLaunchKernelGGL((k_phiu_io<float, true>), grid, block, 0, s, (float*)pu, canon, P, nx, ny, nz);
        else hipLaunchKernelGGL((k_phiu_io<float, false>), grid, block, 0, s, (float*)pu, canon, P, nx, ny, nz);
    }
    return hipGetLastError();
}

hipError_t launch_gamma(int lattice, int precision, const GammaArgs& a, hipStream_t s) {
    const int nbx = (a.nx * a.ny + 255) / 256, nbz = (a.nz + GAMMA_ZB - 1) / GAMMA_ZB;
    const long long nb = (long long)nbx * nbz;
    const dim3 grid((unsigned)nbx, (unsigned)nbz), block(256);
    const bool walls = a.bc[0] != 0 || a.bc[1] != 0 || a.bc[2] != 0;
    auto go_w = [&](auto pair, auto w) {
        using P_ = decltype(pair);
        constexpr int W = decltype(w)::value;
        switch (precision) {
            case 0: hipLaunchKernelGGL((k_gamma_part<P_, 0, W>), grid, block, 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_gamma_part<P_, 1, W>), grid, block, 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_gamma_part<P_, 2, W>), grid, block, 0, s, a); break;
            default: hipLaunchKernelGGL((k_gamma_part<P_, 3, W>), grid, block, 0, s, a);
        }
    };
    auto go = [&](auto pair) {
        if (walls) go_w(pair, std::integral_constant<int, 1>{});
        else go_w(pair, std::integral_constant<int, 0>{});
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gamma_final, dim3(1), dim3(GAMMA_FINAL_THREADS), 0, s, (const double*)a.partials, nb,
                       a.gamma);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nblocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLOCK), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_header(void* dst, const CkHeader& hd, hipStream_t s) {
    hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, (long long*)dst, hd);
    return hipGetLastError();
}

}  // namespace pfk
