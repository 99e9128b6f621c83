// Device code of the fused phase-field lattice Boltzmann time step (gfx950):
// the per-node update, the step kernel and its dispatch over storage forms,
// modes and tiles. Included by kernels.hip (initialisation, I/O, reductions)
// and by step_inst.hip, which instantiates the step kernel for one lattice
// pair and phase-field model per compilation.
//
// One launch = one time step of the coupled solver of Sec. II (hydrodynamics
// of Fakhari2017; phase field: conservative Allen-Cahn of Sec. II.C.1,
// Cahn-Hilliard h-equation of Sec. II.D.1, or the nonlocal / hybrid Allen-Cahn
// of Sec. II.C). Per node, in this order:
//   phi = sum_a h_a                                   (Eq. fakhari_phi_update;
//   nonlocal: phi* + (1 - lam) R / 2, Eq. chai2018_phi_update)
//   grad phi, lap phi from the isotropic central stencils of Sec. III on the
//   hydrodynamic lattice, ghost phi = periodic image or wall mirror
//   rho, nu, tau, mu_phi, p* = sum g, F_s, F_b, F_p   (Eqs. fakhari_rho_update,
//   mu_linear, fakhari_tau_model, chemical_potential, fakhari_p_update, total force)
//   F_mu = nu (grad u + grad u^T) . grad rho with the strain rate from the
//   non-equilibrium second moment of g at u* = sum c g + (F_s+F_b+F_p)/(2 rho)
//   u = sum c g + F/(2 rho)                           (Eq. fakhari_velocity_update)
//   h: BGK with Eqs. fakhari_geq + fakhari_G_modified (AC), liang2_geq +
//   liang2_G with a backward-Euler d(phi u)/dt (CH), or Chai_geq + Hu_G (nonlocal)
//   g: MRT with the stress moments at 1/tau and the rest at s_o, Eqs. fakhari_feq
//   and fakhari_F; in moment space m* = m - S(m - m_eq) + (I - S/2) m_F, which for
//   an orthogonal basis and two rates is
//     g* = g - s_o (g - g_eq) - (1/tau - s_o) P (g - g_eq) + (1 - s_o/2) F_i
//   with P the orthogonal projector on the stress rows (P F_i = 0: F_i is odd
//   in c). P (g - g_eq) needs only the non-equilibrium second moment.
//   streaming: pull between two buffers per distribution (population i of node
//   x is loaded from node x - c_i; halfway bounce-back at walls folded into
//   that load); post-collision values are stored at the node itself.
//
// Layout in HBM: structure of arrays, plane-major [z][q][y][x], planes padded
// to P elements. g storage: float64, float32, or fp16/bf16 of g_i / w_i.
//
// Work decomposition: a workgroup owns a 256-node (x, y) tile (64 x 4, 128 x 2
// or 256 x 1) and marches over zb planes in z. phi of the tile plus a one-node
// halo is rebuilt from h in an LDS ring of four planes; the buffers read this
// step are never written during it, so halo reads of other tiles' nodes are
// race-free.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "lattice.h"

namespace pfk {

// ----------------------------------------------------------------------------
// storage forms

template <int P> struct Types;
template <> struct Types<0> { using T = double; using GS = double;   using HS = double; };
template <> struct Types<1> { using T = float;  using GS = float;    using HS = float;  };
template <> struct Types<2> { using T = float;  using GS = _Float16; using HS = float;  };
template <> struct Types<3> { using T = float;  using GS = uint16_t; using HS = float;  };

// Random words for the stochastic rounding of the 16-bit g store: a
// counter-based generator keyed by the node, the step and the population, so
// the rounding is reproducible and independent of the launch shape. The
// 32-bit integer finaliser "lowbias32" of C. Wellons' hash prospector mixes
// the node index with the mixed step into the seed of a xorshift32 sequence
// (G. Marsaglia, "Xorshift RNGs", J. Stat. Softw. 8(14), 2003). A store takes
// at most 16 random bits (13 for fp16, 16 for bf16), so each word serves two
// populations in a fixed order: its low half, then its high half.
__host__ __device__ constexpr uint32_t sr_mix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
struct SRBits {
    uint32_t s, hi = 0;
    bool have = false;   // hi holds the unused half of the last word
    __device__ __forceinline__ SRBits(uint32_t node, uint32_t step) : s(sr_mix(node ^ sr_mix(step)) | 1u) {}
    // random bits in the low 16 of the result
    __device__ __forceinline__ uint32_t next() {
        if (have) {
            have = false;
            return hi;
        }
        s ^= s << 13;
        s ^= s >> 17;
        s ^= s << 5;
        hi = s >> 16;
        have = true;
        return s;
    }
};

// g codec: the scaled forms store s_i = K g_i / w_i (fp16, K = 4096) or g_i / w_i
// (bf16). enc rounds to nearest even (initialisation, canonical write-back);
// enc_sr, used by the step, rounds stochastically: with r uniform over the
// bits the 16-bit form drops, adding r to the float32 bit pattern and
// truncating rounds the magnitude up with probability equal to the dropped
// fraction of an ulp, so the stored value is unbiased (its expectation is the
// float32 value) and rounding errors do not accumulate systematically over
// steps; the error is below one ulp of the stored form.
template <int P> struct GCodec {
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ T dec(GS v) { return (T)v; }
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ GS enc(T v) { return (GS)v; }
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ GS enc_sr(T v, uint32_t) { return (GS)v; }
};
template <> struct GCodec<2> {
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ float dec(_Float16 v) {
        constexpr float s = (float)(L::w(i) / 4096.0);
        return (float)v * s;
    }
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ _Float16 enc(float v) {
        constexpr float s = (float)(4096.0 / L::w(i));
        return (_Float16)(v * s);
    }
    // 13 float32 mantissa bits below fp16's; the truncated pattern is an fp16
    // value (in fp16's normal range), so the conversion is exact there
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ _Float16 enc_sr(float v, uint32_t r) {
        constexpr float s = (float)(4096.0 / L::w(i));
        const uint32_t b = (__float_as_uint(v * s) + (r & 0x1FFFu)) & 0xFFFFE000u;
        return (_Float16)__uint_as_float(b);
    }
};
template <> struct GCodec<3> {
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ float dec(uint16_t v) {
        constexpr float s = (float)L::w(i);
        return __uint_as_float(((uint32_t)v) << 16) * s;
    }
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ uint16_t enc(float v) {
        constexpr float s = (float)(1.0 / L::w(i));
        uint32_t u = __float_as_uint(v * s);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
    template <class L, int i, class GS, class T>
    static __device__ __forceinline__ uint16_t enc_sr(float v, uint32_t r) {
        constexpr float s = (float)(1.0 / L::w(i));
        return (uint16_t)((__float_as_uint(v * s) + (r & 0xFFFFu)) >> 16);
    }
};

// ----------------------------------------------------------------------------
// index helpers

__device__ __forceinline__ int ghost_coord(int v, int n, int bc) {
    if (bc == 0) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// neighbour x + sgn c_i: linear index, or wall crossing (side 0 low, 1 high)
template <class L, int i, int sgn>
__device__ __forceinline__ bool shifted(int nx, int ny, int nz, const int* bc, int x, int y, int z,
                                        int& idx, int& side) {
    int co[3] = {x, y, z};
    const int n[3] = {nx, ny, nz};
    bool wall = false;
    side = 0;
    unroll<3>([&](auto A) {
        constexpr int ax = A;
        constexpr int d = sgn * L::c(i, ax);
        if constexpr (d != 0) {
            int v = co[ax] + d;
            if (v < 0 || v >= n[ax]) {
                if (bc[ax] == 0) {
                    v = v < 0 ? v + n[ax] : v - n[ax];
                } else {
                    wall = true;
                    side = v < 0 ? 0 : 1;
                }
            }
            co[ax] = v;
        }
    });
    idx = (co[2] * ny + co[1]) * nx + co[0];
    return wall;
}

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    // consecutive workgroup ids go to different XCDs (round robin over 8);
    // give each XCD a contiguous run of tiles so halo rows stay in its L2
    const int per = nb / 8;
    if (bid >= per * 8) return bid;
    return (bid % 8) * per + bid / 8;
}

// ----------------------------------------------------------------------------
// the node update

template <class T>
struct NodeOut {
    T phi, rho, p;
    T u[3];
};

template <class T> __device__ __forceinline__ T rcp(T x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <class T> __device__ __forceinline__ T rsqrt_(T x);
template <> __device__ __forceinline__ float rsqrt_<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsqrt_<double>(double x) { return 1.0 / sqrt(x); }
// 1 / |grad phi| of the interface normal, from s = grad phi . grad phi + eps^2;
// with eps = 0 the guard n = 0 where the gradient vanishes (the antidiffusion
// flux of Eq. fakhari_G_modified then vanishes with it)
template <class T> __device__ __forceinline__ T inv_norm(T s) { return s > (T)0 ? rsqrt_(s) : (T)0; }

// Computes the macroscopic state of one node and, when COLLIDE, hands every
// post-collision population to gsink(i, value) / hsink(a, value) as soon as it
// is formed (so that no array of outputs stays live). Populations are treated
// in opposite pairs (c, -c): equilibria and sources split into a part even in
// c, shared by the pair, and an odd part that changes sign.
// Nonlocal model: source R of the nonlocal AC equation at phi* = sum h (Eq.
// chai_G without its weight) and the phase field phi = phi* + (1 - lam) R / 2
// (Eq. chai2018_phi_update, sum_a G_a = (1 - lam) R). The halo fill and the
// node update evaluate both with these same expressions, so they agree bitwise.
template <class T>
__device__ __forceinline__ T nl_source(const PhysT<T>& ph, T phis, T gam) {
    return ph.mob * (gam * phis * ((T)1 - phis) - ph.w32 * (phis - (T)1) * phis * (phis - (T)0.5));
}
template <class T>
__device__ __forceinline__ T nl_phi(const PhysT<T>& ph, T phis, T gam) {
    return phis + (T)0.5 * ((T)1 - ph.lam) * nl_source(ph, phis, gam);
}

// CH phase-field collision (Eqs. liang2_geq, liang2_G, backward-Euler
// d(phi u)/dt): h* = (1 - 1/tau_phi) h + h_eq / tau_phi + (1 - 1/(2 tau_phi)) G.
// Float forms close each node's phase-field mass balance (sum h* = sum h) on
// the last population: the rounded weights do not sum to one.
template <class HL, class T, class HSink>
__device__ __forceinline__ void ch_collide(const PhysT<T>& ph, const T* h, T phi, const T* u, T mu_phi,
                                           const T* pu_prev, T* pu_new, HSink&& hsink) {
    const T itp = ph.inv_tau_phi, gfp = ph.g_fac_phi;
    const T itp1 = (T)1 - itp;
    T phis = (T)0;
    unroll<HL::Q>([&](auto J) { phis += h[J]; });
    constexpr bool CLOSE = sizeof(T) == 4;
    T hacc = (T)0;
    T pu[3], dpu[3];
    unroll<3>([&](auto A) {
        constexpr int a = A;
        pu[a] = phi * u[a];
        dpu[a] = pu[a] - pu_prev[a];
        pu_new[a] = pu[a];
    });
    const T emu = ph.eta * mu_phi;
    const T v0 = itp1 * h[0] + itp * (phi + ((T)HL::w(0) - (T)1) * emu);
    if constexpr (CLOSE) hacc += v0;
    hsink(std::integral_constant<int, 0>{}, v0);
    unroll<HL::NP>([&](auto K) {
        constexpr int al = HL::pf(K), o = HL::opp(al);
        constexpr T w = (T)HL::w(al);
        constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
        T ep = (T)0, ed = (T)0;
        if constexpr (ex != 0) { ep += (T)ex * pu[0]; ed += (T)ex * dpu[0]; }
        if constexpr (ey != 0) { ep += (T)ey * pu[1]; ed += (T)ey * dpu[1]; }
        if constexpr (ez != 0) { ep += (T)ez * pu[2]; ed += (T)ez * dpu[2]; }
        const T base = itp * w * emu;
        const T t = itp * ((T)3 * w * ep) + gfp * (T)3 * w * ed;
        const T va = itp1 * h[al] + base + t, vo = itp1 * h[o] + base - t;
        if constexpr (CLOSE) hacc += va;
        hsink(std::integral_constant<int, al>{}, va);
        if constexpr (CLOSE && decltype(K)::value == HL::NP - 1) {
            hsink(std::integral_constant<int, o>{}, phis - hacc);
        } else {
            if constexpr (CLOSE) hacc += vo;
            hsink(std::integral_constant<int, o>{}, vo);
        }
    });
}

// Sums below start from their first term, not from zero: 0 + x is not folded
// to x (it differs for x = -0), so a zero start costs one add per sum.
template <bool FIRST, class T>
__device__ __forceinline__ void add_term(T& s, T x) {
    if constexpr (FIRST) s = x;
    else s += x;
}

// first opposite pair (index into L::pf) whose velocity has c_a != 0, or
// c_a c_b != 0 for a != b; -1 if there is none
template <class L>
__host__ __device__ constexpr int first_pair(int a, int b) {
    for (int k = 0; k < L::NP; ++k)
        if ((a == b ? L::c(L::pf(k), a) : L::c(L::pf(k), a) * L::c(L::pf(k), b)) != 0) return k;
    return -1;
}

// c . v for a compile-time velocity c (its nonzero components only)
template <int cx, int cy, int cz, class T>
__device__ __forceinline__ T cdot(const T* v) {
    T r = (T)0;
    if constexpr (cx != 0) r = (T)cx * v[0];
    if constexpr (cy != 0) add_term<cx == 0>(r, (T)cy * v[1]);
    if constexpr (cz != 0) add_term<cx == 0 && cy == 0>(r, (T)cz * v[2]);
    return r;
}

// projection of velocity c on the stress rows, weighted by the row amplitudes:
// 3-D rows 3 c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_y c_z, c_x c_z; 2-D rows
// c_x^2 - c_y^2, c_x c_y
template <int cx, int cy, int cz, bool D3, class T>
__device__ __forceinline__ T stress_proj(T A0, T A1, T Axy, T Ayz, T Axz) {
    constexpr int q0 = D3 ? 3 * cx * cx - (cx * cx + cy * cy + cz * cz) : cx * cx - cy * cy;
    constexpr int q1 = D3 ? cy * cy - cz * cz : 0;
    constexpr int qxy = cx * cy, qyz = D3 ? cy * cz : 0, qxz = D3 ? cx * cz : 0;
    T r = (T)0;
    if constexpr (q0 != 0) r = (T)q0 * A0;
    if constexpr (q1 != 0) add_term<q0 == 0>(r, (T)q1 * A1);
    if constexpr (qxy != 0) add_term<q0 == 0 && q1 == 0>(r, (T)qxy * Axy);
    if constexpr (qyz != 0) add_term<q0 == 0 && q1 == 0 && qxy == 0>(r, (T)qyz * Ayz);
    if constexpr (qxz != 0) add_term<q0 == 0 && q1 == 0 && qxy == 0 && qyz == 0>(r, (T)qxz * Axz);
    return r;
}

// lap phi = 6 sum_i w_i (phi(x + c_i) - phi(x)) over opposite pairs (the same
// order as the node update)
template <class GL, class T>
__device__ __forceinline__ T stencil_lap(const T* phin) {
    const T phi = phin[0];
    T lap = (T)0;
    unroll<GL::NP>([&](auto K) {
        constexpr int k = K;
        constexpr int i = GL::pf(k), o = GL::opp(i);
        add_term<k == 0>(lap, (T)(6.0 * GL::w(i)) * ((phin[i] - phi) + (phin[o] - phi)));
    });
    return lap;
}

// muin: mu_phi at the stencil points (Liang2014 only; the step kernel computes
// it from its phi frame), else unused.
template <class PAIR, int MODEL, class T, bool COLLIDE, class GSink, class HSink>
__device__ __forceinline__ void node_update(const PhysT<T>& ph, const T* g, const T* h, const T* phin,
                                            const T* muin, const T* pu_prev, T* pu_new, NodeOut<T>& mo,
                                            const T gam, GSink&& gsink, HSink&& hsink) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    constexpr bool D3 = PAIR::dim == 3;

    const T phi = phin[0];
    // isotropic stencils: grad = 3 sum w c phi(x+c), lap = 6 sum w (phi(x+c) - phi)
    T gr[3] = {(T)0, (T)0, (T)0};
    T lap = (T)0;
    unroll<GL::NP>([&](auto K) {
        constexpr int k = K;
        constexpr int i = GL::pf(k), o = GL::opp(i);
        const T dp = phin[i] - phin[o];
        unroll<3>([&](auto A) {
            constexpr int a = A;
            if constexpr (GL::c(i, a) != 0)
                add_term<k == first_pair<GL>(a, a)>(gr[a], (T)(3.0 * GL::w(i) * GL::c(i, a)) * dp);
        });
        add_term<k == 0>(lap, (T)(6.0 * GL::w(i)) * ((phin[i] - phi) + (phin[o] - phi)));
    });

    const T dRho = ph.dRho;
    const T rho = ph.rhoL + phi * dRho;
    const T irho = rcp(rho);
    const T nu = ph.visc_mu ? (ph.muL + phi * ph.dMu) * irho : ph.nuL + phi * ph.dNu;
    const T itau = rcp((T)3 * nu + (T)0.5);
    T mu_phi;
    if constexpr (MODEL == 4) mu_phi = muin[0];
    else mu_phi = ph.beta4 * phi * (phi - (T)1) * (phi - (T)0.5) - ph.kappa * lap;

    // moments of g: p*, j, second moment (xx yy zz xy yz xz)
    T ps = g[0];
    T j[3] = {(T)0, (T)0, (T)0};
    T m2[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
    unroll<GL::NP>([&](auto K) {
        constexpr int k = K;
        constexpr int i = GL::pf(k), o = GL::opp(i);
        constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
        const T s = g[i] + g[o], d = g[i] - g[o];
        ps += s;
        if constexpr (cx != 0) { add_term<k == first_pair<GL>(0, 0)>(j[0], (T)cx * d); add_term<k == first_pair<GL>(0, 0)>(m2[0], s); }
        if constexpr (cy != 0) { add_term<k == first_pair<GL>(1, 1)>(j[1], (T)cy * d); add_term<k == first_pair<GL>(1, 1)>(m2[1], s); }
        if constexpr (cz != 0) { add_term<k == first_pair<GL>(2, 2)>(j[2], (T)cz * d); add_term<k == first_pair<GL>(2, 2)>(m2[2], s); }
        if constexpr (cx * cy != 0) add_term<k == first_pair<GL>(0, 1)>(m2[3], (T)(cx * cy) * s);
        if constexpr (cy * cz != 0) add_term<k == first_pair<GL>(1, 2)>(m2[4], (T)(cy * cz) * s);
        if constexpr (cx * cz != 0) add_term<k == first_pair<GL>(0, 2)>(m2[5], (T)(cx * cz) * s);
    });

    if constexpr (MODEL == 4) {
        // ---- Liang2014 hydrodynamics (Sec. II.D.1): F' = F_s + F_a + F_b with
        // F_a = (rho_H - rho_L) M lap(mu_phi) u, u = (sum e f + (F_s + F_b)/2) /
        // (rho - (rho_H - rho_L) M lap(mu_phi) / 2) (Eq. liang2014_velocity_update),
        // p as Eq. liang_p_update; lap(mu_phi) from the mu ring (same stencil as phi)
        const T lapmu = stencil_lap<GL>(muin);
        const T dM = dRho * ph.mob * lapmu;
        const T iden = rcp(rho - (T)0.5 * dM);
        T Fp[3], u[3], grho[3], A[3];
        unroll<3>([&](auto K) {
            constexpr int a = K;
            const T fsb = mu_phi * gr[a] + rho * ph.body[a] + ph.force[a];
            u[a] = (j[a] + (T)0.5 * fsb) * iden;
            Fp[a] = fsb + dM * u[a];
            grho[a] = dRho * gr[a];
            A[a] = (T)(1.0 / 3.0) * grho[a];          // grad(rho c_s^2)
        });
        const T udr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
        const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        constexpr T w0 = (T)GL::w(0);
        const T pres = (T)(1.0 / (3.0 * (1.0 - GL::w(0)))) *
                       ((ps - g[0]) + (T)0.5 * udr - rho * w0 * (T)1.5 * usq);
        mo.phi = phi;
        mo.rho = rho;
        mo.p = pres;
        mo.u[0] = u[0];
        mo.u[1] = u[1];
        mo.u[2] = u[2];
        if constexpr (!COLLIDE) return;

        // ---- f collision: two-rate MRT, f_eq of Eq. liang2_feq, forcing of
        // Eq. liang2_F, F_b = 3 (e - u).[Gamma grad(rho c_s^2) + F' s] with
        // Gamma, s of Eq. Gamma_beta; its traceless second moment is that of
        // B u + u B - 3 (u.B) u u with B = grad(rho c_s^2) + F'
        const T so = ph.s_o;
        const T so1 = (T)1 - so;
        const T dS = itau - so;
        const T fh = (T)1 - (T)0.5 * so;
        const T p3 = (T)3 * pres;
        T B[3];
        unroll<3>([&](auto K) { constexpr int a = K; B[a] = A[a] + Fp[a]; });
        const T uB = u[0] * B[0] + u[1] * B[1] + u[2] * B[2];
        const T uA = u[0] * A[0] + u[1] * A[1] + u[2] * A[2];
        const T uF = u[0] * Fp[0] + u[1] * Fp[1] + u[2] * Fp[2];
        auto pi = [&](int a, int b, T m) {
            return m - rho * u[a] * u[b] + (T)0.5 * (B[a] * u[b] + B[b] * u[a] - (T)3 * uB * u[a] * u[b]);
        };
        const T pxx = pi(0, 0, m2[0]), pyy = pi(1, 1, m2[1]), pzz = pi(2, 2, m2[2]);
        const T pxy = pi(0, 1, m2[3]), pyz = pi(1, 2, m2[4]), pxz = pi(0, 2, m2[5]);
        T A0, A1, Axy, Ayz, Axz;
        if constexpr (D3) {
            A0 = ((T)2 * pxx - pyy - pzz) * (T)StressNorms<GL, 3>::inv_d0;
            A1 = (pyy - pzz) * (T)StressNorms<GL, 3>::inv_d1;
            Axy = pxy * (T)StressNorms<GL, PAIR::dim>::inv_off;
            Ayz = pyz * (T)StressNorms<GL, PAIR::dim>::inv_off;
            Axz = pxz * (T)StressNorms<GL, PAIR::dim>::inv_off;
        } else {
            A0 = (pxx - pyy) * (T)StressNorms<GL, 2>::inv_d0;
            A1 = (T)0;
            Axy = pxy * (T)StressNorms<GL, PAIR::dim>::inv_off;
            Ayz = (T)0;
            Axz = (T)0;
        }
        const T kin0 = rho * (T)(-1.5) * usq;
        const T gam0 = w0 * (T)(-1.5) * usq;
        const T F0 = (T)3 * (-uA * gam0 - uF * (w0 + gam0));
        gsink(std::integral_constant<int, 0>{}, so1 * g[0] + so * (p3 * (w0 - (T)1) + w0 * kin0) + fh * F0);
        unroll<GL::NP>([&](auto K) {
            constexpr int i = GL::pf(K), o = GL::opp(i);
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            constexpr T w = (T)GL::w(i);
            const T cu = cdot<cx, cy, cz>(u), cF = cdot<cx, cy, cz>(Fp), cA = cdot<cx, cy, cz>(A);
            const T P = stress_proj<cx, cy, cz, D3>(A0, A1, Axy, Ayz, Axz);
            const T E = w * (p3 + kin0 + rho * (T)4.5 * cu * cu);
            const T O = w * (T)3 * rho * cu;
            const T Ge = w * ((T)4.5 * cu * cu - (T)1.5 * usq), Go = w * (T)3 * cu;   // Gamma = Ge +/- Go
            const T Fpl = (T)3 * ((cA - uA) * (Ge + Go) + (cF - uF) * (w + Ge + Go));
            const T Fmi = (T)3 * ((-cA - uA) * (Ge - Go) + (-cF - uF) * (w + Ge - Go));
            gsink(std::integral_constant<int, i>{}, so1 * g[i] + so * (E + O) + fh * Fpl - dS * P);
            gsink(std::integral_constant<int, o>{}, so1 * g[o] + so * (E - O) + fh * Fmi - dS * P);
        });
        ch_collide<HL>(ph, h, phi, u, mu_phi, pu_prev, pu_new, hsink);
        return;
    }

    if constexpr (MODEL == 3) {
        // ---- Liang2018 (Sec. II.C): conservative-form hydrodynamics, F = F_s + F_b,
        // rho u = sum e f + F/2 (Eq. liang_velocity_update),
        // p = c_s^2/(1 - w_0) [sum_{b != 0} f + u.grad rho / 2 - rho w_0 u.u/(2 c_s^2)]
        // (Eq. liang_p_update)
        const T irho3 = irho;
        T F[3], u[3], grho[3];
        unroll<3>([&](auto A) {
            constexpr int a = A;
            F[a] = mu_phi * gr[a] + rho * ph.body[a] + ph.force[a];
            u[a] = (j[a] + (T)0.5 * F[a]) * irho3;
            grho[a] = dRho * gr[a];
        });
        const T udr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
        const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        constexpr T w0 = (T)GL::w(0);
        const T pres = (T)(1.0 / (3.0 * (1.0 - GL::w(0)))) *
                       ((ps - g[0]) + (T)0.5 * udr - rho * w0 * (T)1.5 * usq);
        mo.phi = phi;
        mo.rho = rho;
        mo.p = pres;
        mo.u[0] = u[0];
        mo.u[1] = u[1];
        mo.u[2] = u[2];
        if constexpr (!COLLIDE) return;

        // ---- f collision: two-rate MRT with f_eq of Eq. liang_feq and
        // F_b = 3 w [c.F + (c.u)(c.grad rho)] (Eq. liang_F_final, its u.grad rho
        // terms cancel); F has a stress part, so P acts on (f - f_eq) + F / 2:
        // f* = (1 - s_o) f + s_o f_eq + (1 - s_o/2) F - (1/tau - s_o) P (f - f_eq + F/2)
        const T so = ph.s_o;
        const T so1 = (T)1 - so;
        const T dS = itau - so;
        const T fh = (T)1 - (T)0.5 * so;
        const T p3 = (T)3 * pres;                          // p / c_s^2
        // traceless parts of sum c c (f - f_eq) + sum c c F / 2, with
        // sum c c f_eq = p I + rho u u and sum c c F = (u grad rho + grad rho u + (u.grad rho) I) / 3
        auto pi = [&](int a, int b, T m) {
            return m - rho * u[a] * u[b] + (T)(1.0 / 6.0) * (u[a] * grho[b] + u[b] * grho[a]);
        };
        const T pxx = pi(0, 0, m2[0]), pyy = pi(1, 1, m2[1]), pzz = pi(2, 2, m2[2]);
        const T pxy = pi(0, 1, m2[3]), pyz = pi(1, 2, m2[4]), pxz = pi(0, 2, m2[5]);
        T A0, A1, Axy, Ayz, Axz;
        if constexpr (D3) {
            A0 = ((T)2 * pxx - pyy - pzz) * (T)StressNorms<GL, 3>::inv_d0;
            A1 = (pyy - pzz) * (T)StressNorms<GL, 3>::inv_d1;
            Axy = pxy * (T)StressNorms<GL, PAIR::dim>::inv_off;
            Ayz = pyz * (T)StressNorms<GL, PAIR::dim>::inv_off;
            Axz = pxz * (T)StressNorms<GL, PAIR::dim>::inv_off;
        } else {
            A0 = (pxx - pyy) * (T)StressNorms<GL, 2>::inv_d0;
            A1 = (T)0;
            Axy = pxy * (T)StressNorms<GL, PAIR::dim>::inv_off;
            Ayz = (T)0;
            Axz = (T)0;
        }
        const T kin0 = rho * (T)(-1.5) * usq;
        gsink(std::integral_constant<int, 0>{}, so1 * g[0] + so * (p3 * (w0 - (T)1) + w0 * kin0));
        unroll<GL::NP>([&](auto K) {
            constexpr int i = GL::pf(K), o = GL::opp(i);
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            constexpr T w = (T)GL::w(i);
            const T cu = cdot<cx, cy, cz>(u), cf = cdot<cx, cy, cz>(F), cr = cdot<cx, cy, cz>(grho);
            const T P = stress_proj<cx, cy, cz, D3>(A0, A1, Axy, Ayz, Axz);
            const T E = w * (p3 + kin0 + rho * (T)4.5 * cu * cu);   // even part of f_eq
            const T O = w * (T)3 * rho * cu;                         // odd part
            const T Fe = (T)3 * w * cu * cr, Fo = (T)3 * w * cf;     // even / odd parts of F
            const T base = so * E + fh * Fe - dS * P;
            const T t = so * O + fh * Fo;
            gsink(std::integral_constant<int, i>{}, so1 * g[i] + base + t);
            gsink(std::integral_constant<int, o>{}, so1 * g[o] + base - t);
        });

        // ---- h collision: Eqs. liang_geq, liang_G_final,
        // h_eq = w phi (1 + 3 e.u), G = w e.[3 d(phi u)/dt + (4/W) phi (1 - phi) n]
        const T itp = ph.inv_tau_phi, gfp = ph.g_fac_phi;
        const T itp1 = (T)1 - itp;
        constexpr int HOFF = D3 ? 1 : 0;
        T phis = (T)0;
        unroll<HL::Q - HOFF>([&](auto J) { phis += h[J + HOFF]; });
        T pu[3], dpu[3];
        unroll<3>([&](auto A) {
            constexpr int a = A;
            pu[a] = phi * u[a];
            dpu[a] = pu[a] - pu_prev[a];
            pu_new[a] = pu[a];
        });
        const T gg = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        const T coef = ph.anti * phi * ((T)1 - phi) * inv_norm(gg + ph.eps2);
        // float forms close each node's balance on its last population (see below)
        constexpr bool CLOSE = sizeof(T) == 4;
        T hacc = (T)0;
        if constexpr (HL::w(0) != 0.0) {
            const T v = itp1 * h[0] + itp * (T)HL::w(0) * phi;
            if constexpr (CLOSE) hacc += v;
            hsink(std::integral_constant<int, 0>{}, v);
        }
        unroll<HL::NP>([&](auto K) {
            constexpr int al = HL::pf(K), o = HL::opp(al);
            constexpr T w = (T)HL::w(al);
            constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
            T eu = (T)0, eg = (T)0, ed = (T)0;
            if constexpr (ex != 0) { eu += (T)ex * u[0]; eg += (T)ex * gr[0]; ed += (T)ex * dpu[0]; }
            if constexpr (ey != 0) { eu += (T)ey * u[1]; eg += (T)ey * gr[1]; ed += (T)ey * dpu[1]; }
            if constexpr (ez != 0) { eu += (T)ez * u[2]; eg += (T)ez * gr[2]; ed += (T)ez * dpu[2]; }
            const T base = itp * w * phi;
            const T t = itp * ((T)3 * w * phi * eu) + gfp * w * ((T)3 * ed + coef * eg);
            const T va = itp1 * h[al] + base + t, vo = itp1 * h[o] + base - t;
            if constexpr (CLOSE) hacc += va;
            hsink(std::integral_constant<int, al>{}, va);
            if constexpr (CLOSE && decltype(K)::value == HL::NP - 1) {
                hsink(std::integral_constant<int, o>{}, phis - hacc);
            } else {
                if constexpr (CLOSE) hacc += vo;
                hsink(std::integral_constant<int, o>{}, vo);
            }
        });
        return;
    }

    // forces: F_s + F_b + F_p, with F_p = -(p/rho) grad rho = -c_s^2 p* dRho grad phi
    const T inv2rho = (T)0.5 * irho;
    const T sg = mu_phi - ps * dRho * (T)(1.0 / 3.0);
    T F[3];
    unroll<3>([&](auto A) {
        constexpr int a = A;
        F[a] = sg * gr[a] + rho * ph.body[a] + ph.force[a];
    });
    // strain from the non-equilibrium second moment at u* (sum c c g_eq = p*/3 I + u u)
    T us[3];
    unroll<3>([&](auto A) { constexpr int a = A; us[a] = j[a] + F[a] * inv2rho; });
    const T s3 = ps * (T)(1.0 / 3.0);
    const T sfac = (T)(-3.0) * itau;            // S = -Pi / (tau c_s^2)
    T S[6];
    S[0] = sfac * (m2[0] - s3 - us[0] * us[0]);
    S[1] = sfac * (m2[1] - s3 - us[1] * us[1]);
    S[2] = D3 ? sfac * (m2[2] - s3 - us[2] * us[2]) : (T)0;
    S[3] = sfac * (m2[3] - us[0] * us[1]);
    S[4] = D3 ? sfac * (m2[4] - us[1] * us[2]) : (T)0;
    S[5] = D3 ? sfac * (m2[5] - us[0] * us[2]) : (T)0;
    const T nr = nu * dRho;                     // F_mu = nu S . grad rho
    F[0] += nr * (S[0] * gr[0] + S[3] * gr[1] + S[5] * gr[2]);
    F[1] += nr * (S[3] * gr[0] + S[1] * gr[1] + S[4] * gr[2]);
    F[2] += nr * (S[5] * gr[0] + S[4] * gr[1] + S[2] * gr[2]);
    T u[3];
    unroll<3>([&](auto A) { constexpr int a = A; u[a] = j[a] + F[a] * inv2rho; });

    mo.phi = phi;
    mo.rho = rho;
    mo.p = rho * s3;
    mo.u[0] = u[0];
    mo.u[1] = u[1];
    mo.u[2] = u[2];
    if constexpr (!COLLIDE) return;

    // ---- g collision (two-rate MRT, projector form)
    const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T so = ph.s_o;
    const T so1 = (T)1 - so;
    const T dS = itau - so;
    const T ffac = ((T)1 - (T)0.5 * so) * (T)3 * irho;
    const T aeq = ps - (T)1.5 * usq;
    // non-equilibrium second moment at the final u
    const T pxx = m2[0] - s3 - u[0] * u[0], pyy = m2[1] - s3 - u[1] * u[1];
    const T pzz = m2[2] - s3 - u[2] * u[2];
    const T pxy = m2[3] - u[0] * u[1], pyz = m2[4] - u[1] * u[2], pxz = m2[5] - u[0] * u[2];
    T A0, A1, Axy, Ayz, Axz;
    if constexpr (D3) {
        // projections on the stress rows 3cx^2 - c^2, cy^2 - cz^2, cx cy, cy cz, cx cz
        A0 = ((T)2 * pxx - pyy - pzz) * (T)StressNorms<GL, 3>::inv_d0;
        A1 = (pyy - pzz) * (T)StressNorms<GL, 3>::inv_d1;
        Axy = pxy * (T)StressNorms<GL, PAIR::dim>::inv_off;
        Ayz = pyz * (T)StressNorms<GL, PAIR::dim>::inv_off;
        Axz = pxz * (T)StressNorms<GL, PAIR::dim>::inv_off;
    } else {
        // stress rows cx^2 - cy^2 and cx cy
        A0 = (pxx - pyy) * (T)StressNorms<GL, 2>::inv_d0;
        A1 = (T)0;
        Axy = pxy * (T)StressNorms<GL, PAIR::dim>::inv_off;
        Ayz = (T)0;
        Axz = (T)0;
    }
    // rest population: no odd part, no stress projection
    gsink(std::integral_constant<int, 0>{}, so1 * g[0] + so * (T)GL::w(0) * aeq);
    unroll<GL::NP>([&](auto K) {
        constexpr int i = GL::pf(K), o = GL::opp(i);
        constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
        constexpr T w = (T)GL::w(i);
        const T cu = cdot<cx, cy, cz>(u), cf = cdot<cx, cy, cz>(F);
        const T P = stress_proj<cx, cy, cz, D3>(A0, A1, Axy, Ayz, Axz);
        // g_eq = E +/- O with E = w (aeq + 4.5 (c.u)^2), O = 3 w c.u; F_i = +/- w c.F ...
        const T E = w * (aeq + (T)4.5 * cu * cu);
        const T base = so * E - dS * P;
        const T t = so * ((T)3 * w * cu) + ffac * w * cf;
        gsink(std::integral_constant<int, i>{}, so1 * g[i] + base + t);
        gsink(std::integral_constant<int, o>{}, so1 * g[o] + base - t);
    });

    // ---- h collision (BGK): h* = (1 - 1/tau_phi) h + h_eq / tau_phi + (1 - 1/(2 tau_phi)) G
    const T itp = ph.inv_tau_phi, gfp = ph.g_fac_phi;
    const T itp1 = (T)1 - itp;
    // phi* = sum h, in the order of the halo fill
    constexpr int HOFF = rest_offset(MODEL, D3);
    T phis = (T)0;
    unroll<HL::Q - HOFF>([&](auto J) { phis += h[J + HOFF]; });
    // Float forms: the rounded weights do not sum to one (6 fl(1/6) = 1 + 3e-8),
    // which would add a fixed fraction of phi to the phase-field mass every
    // step. There the last population closes the node's exact balance instead:
    // sum_a h*_a = phi* + (1/(2 tau_phi) + 1 - 1/(2 tau_phi)) sum_a G_a, where
    // sum_a G_a = (1 - lam) R for the nonlocal model and 0 otherwise.
    constexpr bool CLOSE = sizeof(T) == 4;
    T hacc = (T)0, htarget = phis;
    auto put = [&](auto J, T v) {
        if constexpr (CLOSE) hacc += v;
        hsink(J, v);
    };
    auto put_pair = [&](auto K, auto A, auto O, T va, T vo) {
        put(A, va);
        if constexpr (CLOSE && decltype(K)::value == HL::NP - 1) hsink(O, htarget - hacc);
        else put(O, vo);
    };
    if constexpr (MODEL == 0) {
        const T gg = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        const T coef = ph.anti * phi * ((T)1 - phi) * inv_norm(gg + ph.eps2);
        const T e0 = phi * ((T)1 - (T)1.5 * usq);
        if constexpr (HL::w(0) != 0.0)
            put(std::integral_constant<int, 0>{}, itp1 * h[0] + itp * (T)HL::w(0) * e0);
        unroll<HL::NP>([&](auto K) {
            constexpr int al = HL::pf(K), o = HL::opp(al);
            constexpr T w = (T)HL::w(al);
            constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
            T eu = (T)0, eg = (T)0;
            if constexpr (ex != 0) { eu += (T)ex * u[0]; eg += (T)ex * gr[0]; }
            if constexpr (ey != 0) { eu += (T)ey * u[1]; eg += (T)ey * gr[1]; }
            if constexpr (ez != 0) { eu += (T)ez * u[2]; eg += (T)ez * gr[2]; }
            const T base = itp * w * (e0 + (T)4.5 * phi * eu * eu);
            const T t = itp * ((T)3 * w * phi * eu) + gfp * w * coef * eg;
            put_pair(K, std::integral_constant<int, al>{}, std::integral_constant<int, o>{},
                     itp1 * h[al] + base + t, itp1 * h[o] + base - t);
        });
    } else if constexpr (MODEL == 2) {
        // Eqs. Chai_geq, Hu_G: h_eq = w phi (1 + e.u / c_s^2),
        // G = lam w e.[(4/W) phi (1 - phi) n] + (1 - lam) w R, R at phi* = sum h
        const T R = nl_source(ph, phis, gam);
        htarget = phis + ((T)1 - ph.lam) * ((T)0.5 * itp + gfp) * R;
        const T gg = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        const T coef = ph.anti * phi * ((T)1 - phi) * inv_norm(gg + ph.eps2);
        const T gcon = gfp * ph.lam * coef;
        const T giso = gfp * ((T)1 - ph.lam) * R;
        const T e0 = itp * phi + giso;
        if constexpr (HL::w(0) != 0.0)
            put(std::integral_constant<int, 0>{}, itp1 * h[0] + (T)HL::w(0) * e0);
        unroll<HL::NP>([&](auto K) {
            constexpr int al = HL::pf(K), o = HL::opp(al);
            constexpr T w = (T)HL::w(al);
            constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
            T eu = (T)0, eg = (T)0;
            if constexpr (ex != 0) { eu += (T)ex * u[0]; eg += (T)ex * gr[0]; }
            if constexpr (ey != 0) { eu += (T)ey * u[1]; eg += (T)ey * gr[1]; }
            if constexpr (ez != 0) { eu += (T)ez * u[2]; eg += (T)ez * gr[2]; }
            const T base = w * e0;
            const T t = itp * ((T)3 * w * phi * eu) + gcon * w * eg;
            put_pair(K, std::integral_constant<int, al>{}, std::integral_constant<int, o>{},
                     itp1 * h[al] + base + t, itp1 * h[o] + base - t);
        });
    } else {
        ch_collide<HL>(ph, h, phi, u, mu_phi, pu_prev, pu_new, hsink);
    }
}

// ----------------------------------------------------------------------------
// block reduction of the diagnostics (fixed order, deterministic)

struct DiagAcc {
    double v[NDIAG];
};

__device__ __forceinline__ void diag_init(DiagAcc& d) {
    for (int k = 0; k < NDIAG; ++k) d.v[k] = 0.0;
    d.v[3] = 1e300;    // phi_min
    d.v[4] = -1e300;   // phi_max
}

__device__ __forceinline__ void diag_combine(double* a, const double* b) {
    for (int k = 0; k < NDIAG; ++k) {
        if (k == 3) a[k] = fmin(a[k], b[k]);
        else if (k == 4 || k == 5 || k == 10) a[k] = fmax(a[k], b[k]);
        else a[k] += b[k];
    }
}

__device__ void block_reduce_diag(DiagAcc& d, double* out) {
    __shared__ double red[BLOCK / 64][NDIAG];
    for (int off = 32; off >= 1; off >>= 1) {
        double o[NDIAG];
        for (int k = 0; k < NDIAG; ++k) o[k] = __shfl_xor(d.v[k], off, 64);
        diag_combine(d.v, o);
    }
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    if (lane == 0)
        for (int k = 0; k < NDIAG; ++k) red[wv][k] = d.v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc[NDIAG];
        for (int k = 0; k < NDIAG; ++k) acc[k] = red[0][k];
        for (int w = 1; w < BLOCK / 64; ++w) diag_combine(acc, red[w]);
        for (int k = 0; k < NDIAG; ++k) out[k] = acc[k];
    }
}

// ----------------------------------------------------------------------------
// fused step kernel

// Element index helpers for the plane-major layout [z][q][y][x].
template <int Q>
__device__ __forceinline__ size_t el(int z, int q, int inplane, int P) {
    return ((size_t)z * Q + q) * (size_t)P + (unsigned)inplane;
}

// element inplane of population plane (z, q): a uniform plane base plus a
// 32-bit byte offset, so loads and stores take the scalar-base addressing form
template <int Q, class E>
__device__ __forceinline__ E& at(E* arr, int z, int q, int P, int inplane) {
    E* base = arr + ((size_t)z * Q + q) * (size_t)P;
    return *(E*)((char*)base + (size_t)((unsigned)inplane * (unsigned)sizeof(E)));
}
template <int Q, class E>
__device__ __forceinline__ const E& at(const E* arr, int z, int q, int P, int inplane) {
    const E* base = arr + ((size_t)z * Q + q) * (size_t)P;
    return *(const E*)((const char*)base + (size_t)((unsigned)inplane * (unsigned)sizeof(E)));
}

// Hide a per-lane offset from loop-invariant code motion. In the z march every
// load and store addresses a uniform plane base (scalar registers) plus a
// 32-bit lane offset that does not change along the column; seen as invariant,
// base + offset is hoisted into a 64-bit per-lane pointer and every access
// then pays a 64-bit vector add (and two registers per pointer). Marking the
// offset as redefined each plane keeps the scalar-base addressing form.
__device__ __forceinline__ void lane_opaque(int& v) { asm volatile("" : "+v"(v)); }

// Geometry of the column (x, y) a thread owns for the whole z march: in-plane
// offsets of the 3 x 3 neighbourhood with the periodic wrap folded in (the
// wall side keeps the node itself), and wall flags of the x and y neighbours.
struct Column {
    int off[3][3];       // [dy + 1][dx + 1] -> (y + dy) * nx + (x + dx), wrapped
    bool wx[2], wy[2];   // the x / y neighbour at -1 / +1 lies beyond a wall
};

__device__ __forceinline__ void axis_nb(int v, int n, int bc, int* o, bool* w) {
    const bool lo = v == 0, hi = v == n - 1;
    o[0] = lo ? (bc == 0 ? n - 1 : 0) : v - 1;
    o[1] = v;
    o[2] = hi ? (bc == 0 ? 0 : n - 1) : v + 1;
    w[0] = lo && bc != 0;
    w[1] = hi && bc != 0;
}

// z planes of the neighbourhood of plane z (wrapped; clamped at a wall) and
// wall flags, uniform over the workgroup
struct ZPlanes {
    int zk[3];
    bool wz[2];
};

// does x + sgn c_i lie beyond a wall; which side
template <class L, int i, int sgn>
__device__ __forceinline__ bool beyond(const Column& cl, const ZPlanes& zp, int& side) {
    constexpr int cx = sgn * L::c(i, 0), cy = sgn * L::c(i, 1), cz = sgn * L::c(i, 2);
    bool w = false;
    side = 0;
    if constexpr (cx != 0) { const bool f = cl.wx[cx > 0]; w = w || f; side = f ? (cx > 0) : side; }
    if constexpr (cy != 0) { const bool f = cl.wy[cy > 0]; w = w || f; side = f ? (cy > 0) : side; }
    if constexpr (cz != 0) { const bool f = zp.wz[cz > 0]; w = w || f; side = f ? (cz > 0) : side; }
    return w;
}

// In-plane offset of a node and of its four axis neighbours (wrapped; the
// node itself on a wall side), with the wall flags of those neighbours.
struct Cross {
    int c, xm, xp, ym, yp;
    bool wxm, wxp, wym, wyp;
};

__device__ __forceinline__ void lane_opaque(Cross& X) {
    lane_opaque(X.c);
    lane_opaque(X.xm);
    lane_opaque(X.xp);
    lane_opaque(X.ym);
    lane_opaque(X.yp);
}

__device__ __forceinline__ Cross make_cross(int px, int py, int nx, int ny, const int* bc) {
    int ox[3], oy[3];
    bool wx[2], wy[2];
    axis_nb(px, nx, bc[0], ox, wx);
    axis_nb(py, ny, bc[1], oy, wy);
    Cross X;
    X.c = py * nx + px;
    X.xm = py * nx + ox[0];
    X.xp = py * nx + ox[2];
    X.ym = oy[0] * nx + px;
    X.yp = oy[2] * nx + px;
    X.wxm = wx[0];
    X.wxp = wx[1];
    X.wym = wy[0];
    X.wyp = wy[1];
    return X;
}

__device__ __forceinline__ ZPlanes make_zplanes(int z, int nz, int bc) {
    ZPlanes zp;
    int oz[3];
    axis_nb(z, nz, bc, oz, zp.wz);
    zp.zk[0] = oz[0];
    zp.zk[1] = oz[1];
    zp.zk[2] = oz[2];
    return zp;
}

// Post-streaming phase-field population al at the node of X in plane zp.zk[1]:
// pulled from the node x - e_al of the previous step's post-collision buffer,
// or, if that node lies beyond a wall, the bounce-back of slot opp(al) here.
// D3Q7 / D2Q5 velocities are axis-aligned: one component at most is nonzero.
template <class HL, int al, int HOFF, int WALLS, class T, class HS>
__device__ __forceinline__ T pull_h(const HS* __restrict__ H, const Cross& X, const ZPlanes& zp, int P) {
    constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
    constexpr int QS = HL::Q - HOFF;
    const int off = ex > 0 ? X.xm : (ex < 0 ? X.xp : (ey > 0 ? X.ym : (ey < 0 ? X.yp : X.c)));
    if constexpr (WALLS) {
        const bool w = (ex > 0 && X.wxm) || (ex < 0 && X.wxp) || (ey > 0 && X.wym) || (ey < 0 && X.wyp) ||
                       (ez > 0 && zp.wz[0]) || (ez < 0 && zp.wz[1]);
        constexpr int o = HL::opp(al);
        const size_t e = w ? el<QS>(zp.zk[1], o - HOFF, X.c, P) : el<QS>(zp.zk[1 - ez], al - HOFF, off, P);
        return (T)H[e];
    } else {
        return (T)at<QS>(H, zp.zk[1 - ez], al - HOFF, P, off);
    }
}

// WALLS = 0: every axis periodic (no bounce-back selects are compiled).
// TS: tile shape, TX x TY nodes per workgroup of NT threads (one node each):
// 0 = 64 x 4 and 3 = 256 x 4 (1024 threads) with workgroups ordered so each
// XCD sweeps a contiguous run of tiles, 1 = 128 x 2 and 2 = 256 x 1 in
// hardware order.
template <class PAIR, int MODEL, int PREC, int MODE, int WALLS, int TS>
__global__ __launch_bounds__(TILE_THREADS[TS]) void k_step(const KArgs a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    using T = typename Types<PREC>::T;
    using GS = typename Types<PREC>::GS;
    using HS = typename Types<PREC>::HS;
    using GC = GCodec<PREC>;
    constexpr int QG = GL::Q, QH = HL::Q;
    constexpr bool D3 = PAIR::dim == 3;
    constexpr int HOFF = rest_offset(MODEL, D3);        // zero-weight D3Q7 rest population not stored
    constexpr int QHS = QH - HOFF;
    constexpr int NT = TILE_THREADS[TS];
    constexpr int TX = TILE_NX[TS], TY = TILE_NY[TS];
    static_assert(TX * TY == NT, "one node per thread");
    // Liang2014 needs mu_phi at the stencil points: computed here from phi, on
    // the tile and a halo of one, so its phi frame reaches two nodes out
    constexpr bool MUF = MODEL == 4;
    constexpr int RH = MUF ? 2 : 1;                    // halo of the phi frame
    constexpr int PW = TX + 2 * RH, PSZ = PW * (TY + 2 * RH);
    constexpr int NRING = PSZ - TX * TY;               // halo positions of the frame
    constexpr int ZL = MUF ? 2 : 1;                    // phi planes filled ahead of the node plane
    constexpr int NPL = D3 ? (MUF ? 5 : 4) : 1;        // phi planes held (ring)
    __shared__ T lphi[NPL * PSZ];
    constexpr int MW = TX + 2, MSZ = MW * (TY + 2);    // mu frame
    constexpr int NMU = MUF ? (MSZ + NT - 1) / NT : 1; // mu positions per thread
    __shared__ T lmu[MUF ? (D3 ? 4 : 1) * MSZ : 1];

    const int b = (TS == 0 || TS >= 3) ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int bx = b % a.ntx, byz = b / a.ntx;
    const int by = byz % a.nty, bz = byz / a.nty;
    const int x0 = bx * TX, y0 = by * TY;
    const int zs = bz * a.zb;
    const int ze = min(a.nz, zs + a.zb);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = x < a.nx && y < a.ny;
    const int nx = a.nx, ny = a.ny, nz = a.nz, P = a.P;
    const GS* __restrict__ Gin = (const GS*)a.gin;
    GS* __restrict__ Gout = (GS*)a.gout;
    const HS* __restrict__ Hin = (const HS*)a.hin;
    HS* __restrict__ Hout = (HS*)a.hout;
    T* __restrict__ PU = (T*)a.phiu;

    const PhysT<T>* php;
    if constexpr (sizeof(T) == 8) php = &a.ph;
    else php = &a.phf;
    const PhysT<T>& ph = *php;
    T gam = (T)0;                    // nonlocal multiplier of this step
    if constexpr (MODEL == 2) gam = (T)*a.gamma;
    auto gcorr = [&](int side, int i) -> T {
        if constexpr (sizeof(T) == 8) return a.gcorr[side][i];
        else return a.gcorrf[side][i];
    };

    // the thread's own tile position, wrapped or clamped (inactive threads fill
    // the halo of the domain edge with it)
    Cross ocr = make_cross(ghost_coord(x, nx, a.bc[0]), ghost_coord(y, ny, a.bc[1]), nx, ny, a.bc);
    Column cl;
    {
        int ox[3], oy[3];
        axis_nb(min(x, nx - 1), nx, a.bc[0], ox, cl.wx);
        axis_nb(min(y, ny - 1), ny, a.bc[1], oy, cl.wy);
        for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) cl.off[dy][dx] = oy[dy] * nx + ox[dx];
    }
    // halo ring positions this thread fills (ring index threadIdx.x + k NT)
    constexpr int NR = (NRING + NT - 1) / NT;
    Cross rcr[NR];
    int ring_lds[NR];
    bool ring[NR];
    for (int k = 0; k < NR; ++k) {
        const int r = threadIdx.x + k * NT;
        ring[k] = r < NRING;
        int hx = 0, hy = 0;
        // RH rows above, RH rows below, then RH columns left and right
        if (r < RH * PW) { hy = r / PW - RH; hx = r % PW - RH; }
        else if (r < 2 * RH * PW) { const int q = r - RH * PW; hy = TY + q / PW; hx = q % PW - RH; }
        else if (r < 2 * RH * PW + RH * TY) { const int q = r - 2 * RH * PW; hx = q / TY - RH; hy = q % TY; }
        else { const int q = r - 2 * RH * PW - RH * TY; hx = TX + q / TY; hy = q % TY; }
        if (!ring[k]) { hx = 0; hy = 0; }
        rcr[k] = make_cross(ghost_coord(x0 + hx, nx, a.bc[0]), ghost_coord(y0 + hy, ny, a.bc[1]), nx, ny, a.bc);
        ring_lds[k] = (hy + RH) * PW + (hx + RH);
    }
    const int own_lds = (ly + RH) * PW + (lx + RH);
    // phi ring slot of plane zz (zz >= zs - ZL) and mu ring slot (zz >= zs - 1)
    auto phi_slot = [&](int zz) { return D3 ? (zz - zs + ZL) % NPL : 0; };
    auto mu_slot = [&](int zz) { return D3 ? (zz - zs + 1) & 3 : 0; };
    // mu positions this thread computes (mu-frame index threadIdx.x + m NT) and
    // the phi-frame position of each one's stencil centre: the position itself,
    // or beyond an x / y wall the clamped node inside (a ghost takes the mu_phi
    // of the node it mirrors, as a ghost phi takes its phi)
    int mu_c[NMU];
    bool mu_on[NMU];
    if constexpr (MUF) {
        for (int m = 0; m < NMU; ++m) {
            const int q = threadIdx.x + m * NT;
            mu_on[m] = q < MSZ;
            const int mx = (mu_on[m] ? q % MW : 1) - 1, my = (mu_on[m] ? q / MW : 1) - 1;
            int cxp = mx, cyp = my;
            if (a.bc[0] != 0) cxp = min(max(x0 + mx, 0), nx - 1) - x0;
            if (a.bc[1] != 0) cyp = min(max(y0 + my, 0), ny - 1) - y0;
            mu_c[m] = (cyp + RH) * PW + (cxp + RH);
        }
    }

    DiagAcc acc;
    if constexpr (MODE == MODE_DIAG) diag_init(acc);

    // phi of plane zz into LDS slot; returns the thread's own h of that plane.
    // phi = sum of the post-streaming h, pulled from the previous step's buffer.
    T hn[QH];
    auto fill_plane = [&](int zz, int slot) {
        const int zu = __builtin_amdgcn_readfirstlane(zz);
        const ZPlanes fz = make_zplanes(D3 ? ghost_coord(zu, nz, a.bc[2]) : 0, nz, a.bc[2]);
        // every load of the plane first (ring loads unconditional: a thread with
        // no ring position reads a valid in-tile node and discards it), then the
        // sums, so the loads overlap instead of waiting on each other
        T rv[NR][QHS];
        hn[0] = (T)0;
        unroll<QHS>([&](auto J) {
            constexpr int al = J + HOFF;
            hn[al] = pull_h<HL, al, HOFF, WALLS, T>(Hin, ocr, fz, P);
        });
        for (int k = 0; k < NR; ++k)
            unroll<QHS>([&](auto J) {
                constexpr int al = J + HOFF;
                rv[k][J] = pull_h<HL, al, HOFF, WALLS, T>(Hin, rcr[k], fz, P);
            });
        T s = (T)0;
        unroll<QHS>([&](auto J) {
            constexpr int al = J + HOFF;
            s += hn[al];
        });
        if constexpr (MODEL == 2) s = nl_phi(ph, s, gam);
        lphi[slot * PSZ + own_lds] = s;
        for (int k = 0; k < NR; ++k) {
            T sr = (T)0;
            unroll<QHS>([&](auto J) { sr += rv[k][J]; });
            if constexpr (MODEL == 2) sr = nl_phi(ph, sr, gam);
            if (ring[k]) lphi[slot * PSZ + ring_lds[k]] = sr;
        }
    };

    // Liang2014: mu_phi of plane zz on the mu frame, from the phi ring, with the
    // stencil and expression of the chemical potential at a node; beyond a z
    // wall the stencil is centred on the plane inside
    auto fill_mu = [&](int zz) {
        int zc = zz;
        if constexpr (D3) {
            if (a.bc[2] != 0) zc = min(max(zz, 0), nz - 1);
        }
        const T* pm = lphi + phi_slot(zc - 1) * PSZ;
        const T* p0 = lphi + phi_slot(zc) * PSZ;
        const T* pp = lphi + phi_slot(zc + 1) * PSZ;
        T* mo_ = lmu + mu_slot(zz) * MSZ;
        for (int m = 0; m < NMU; ++m) {
            T phin[QG];
            unroll<QG>([&](auto I) {
                constexpr int i = I;
                constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
                const T* pl_ = cz < 0 ? pm : (cz > 0 ? pp : p0);
                phin[i] = pl_[mu_c[m] + cy * PW + cx];
            });
            const T phi = phin[0];
            const T lap = stencil_lap<GL>(phin);
            if (mu_on[m])
                mo_[threadIdx.x + m * NT] = ph.beta4 * phi * (phi - (T)1) * (phi - (T)0.5) - ph.kappa * lap;
        }
    };

    // stored g that the pull of plane z reads (storage form, not decoded)
    auto pull_g = [&](int z, GS* gr) {
        const ZPlanes zp = make_zplanes(z, nz, a.bc[2]);
        const int o11 = cl.off[1][1];
        unroll<QG>([&](auto I) {
            constexpr int i = I;
            constexpr int o = GL::opp(i);
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            if constexpr (!WALLS) {
                gr[i] = at<QG>(Gin, zp.zk[1 - cz], i, P, cl.off[1 - cy][1 - cx]);
            } else {
                int side;
                // beyond a wall: the bounce-back of what left this node, slot opp(i)
                const bool w = beyond<GL, i, -1>(cl, zp, side);
                gr[i] = Gin[w ? el<QG>(z, o, o11, P) : el<QG>(zp.zk[1 - cz], i, cl.off[1 - cy][1 - cx], P)];
            }
        });
    };

    // node update of plane z: slots sm, s0, sp hold planes z - 1, z, z + 1
    auto do_node = [&](int z, const GS* gr, const T* h, int sm, int s0, int sp) {
        const T* pm = lphi + sm * PSZ;
        const T* p0 = lphi + s0 * PSZ;
        const T* pp = lphi + sp * PSZ;
        const int o11 = cl.off[1][1];
        const ZPlanes zp = make_zplanes(z, nz, a.bc[2]);
        // post-streaming g of this node (pulled from x - c_i), decoded
        T g[QG];
        unroll<QG>([&](auto I) {
            constexpr int i = I;
            g[i] = GC::template dec<GL, i, GS, T>(gr[i]);   // w_opp(i) = w_i: same codec
            if constexpr (WALLS) {
                int side;
                if (beyond<GL, i, -1>(cl, zp, side)) g[i] += gcorr(side, GL::opp(i));
            }
        });
        T pu_prev[3] = {(T)0, (T)0, (T)0};
        if constexpr (MODEL == 1 || MODEL == 3 || MODEL == 4) {
            unroll<3>([&](auto A) {
                constexpr int c = A;
                pu_prev[c] = at<3>(PU, z, c, P, o11);
            });
        }
        // phi (and, for Liang2014, mu_phi) at the stencil points
        T phin[QG];
        T muin[MUF ? QG : 1];
        unroll<QG>([&](auto I) {
            constexpr int i = I;
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            const int sl = cz < 0 ? sm : (cz > 0 ? sp : s0);
            phin[i] = lphi[sl * PSZ + (ly + RH + cy) * PW + (lx + RH + cx)];
            if constexpr (MUF) muin[i] = lmu[mu_slot(z + cz) * MSZ + (ly + 1 + cy) * MW + (lx + 1 + cx)];
        });
        NodeOut<T> mo;
        T pu_new[3];
        if constexpr (MODE == MODE_RECORD) {
            // the state this step starts from, as the canonical read-out forms it
            const size_t nn = (size_t)nx * ny * nz;
            const size_t idx = ((size_t)z * ny + y) * nx + x;
            if (a.xf32) {
                unroll<QG>([&](auto I) { constexpr int i = I; ((float*)a.xg)[i * nn + idx] = (float)g[i]; });
                unroll<QH>([&](auto J) { constexpr int al = J; ((float*)a.xh)[al * nn + idx] = (float)h[al]; });
            } else {
                unroll<QG>([&](auto I) { constexpr int i = I; ((double*)a.xg)[i * nn + idx] = (double)g[i]; });
                unroll<QH>([&](auto J) { constexpr int al = J; ((double*)a.xh)[al * nn + idx] = (double)h[al]; });
            }
            if constexpr (MODEL == 1 || MODEL == 3 || MODEL == 4) {
                if (a.xpu) {
                    if (a.xf32)
                        unroll<3>([&](auto A) { constexpr int c = A; ((float*)a.xpu)[c * nn + idx] = (float)pu_prev[c]; });
                    else
                        unroll<3>([&](auto A) { constexpr int c = A; ((double*)a.xpu)[c * nn + idx] = (double)pu_prev[c]; });
                }
            }
        }
        if constexpr (MODE == MODE_STEP || MODE == MODE_RECORD) {
            // post-collision populations at the node itself, in the other buffers;
            // streamed (non-temporal stores): no workgroup reads them this step.
            // The store offset is opaque here too, or one 64-bit lane pointer is
            // formed and every store adds its plane base to it in vector code.
            int so = o11;
            lane_opaque(so);
            // Liang2014 keeps round-to-nearest: its 1024-thread kernel sits at
            // 118 of its 128 registers, and the stochastic rounding pushes it
            // over (spills, 16 % slower)
            SRBits rb((uint32_t)(((size_t)z * ny + y) * nx + x), a.step);
            auto gsink = [&](auto I, T v) {
                constexpr int i = I;
                if constexpr (MODEL == 4)
                    __builtin_nontemporal_store(GC::template enc<GL, i, GS, T>(v), &at<QG>(Gout, z, i, P, so));
                else
                    __builtin_nontemporal_store(GC::template enc_sr<GL, i, GS, T>(v, rb.next()), &at<QG>(Gout, z, i, P, so));
            };
            auto hsink = [&](auto J, T v) {
                constexpr int al = J;
                if constexpr (al >= HOFF) {
                    if (a.write_h) __builtin_nontemporal_store((HS)v, &at<QHS>(Hout, z, al - HOFF, P, so));
                }
            };
            node_update<PAIR, MODEL, T, true>(ph, g, h, phin, muin, pu_prev, pu_new, mo, gam, gsink, hsink);
            if constexpr (MODEL == 1 || MODEL == 3 || MODEL == 4) {
                if (a.write_h) {
                    unroll<3>([&](auto A) {
                        constexpr int c = A;
                        at<3>(PU, z, c, P, o11) = pu_new[c];
                    });
                }
            }
        } else {
            auto none = [](auto, T) {};
            node_update<PAIR, MODEL, T, false>(ph, g, h, phin, muin, pu_prev, pu_new, mo, gam, none, none);
            const size_t idx = ((size_t)z * ny + y) * nx + x;    // canonical index
            if constexpr (MODE == MODE_FIELDS) {
                if (a.f_phi) a.f_phi[idx] = (double)mo.phi;
                if (a.f_rho) a.f_rho[idx] = (double)mo.rho;
                if (a.f_p) a.f_p[idx] = (double)mo.p;
                if (a.f_u) {
                    const size_t nn = (size_t)nx * ny * nz;
                    a.f_u[idx] = (double)mo.u[0];
                    a.f_u[nn + idx] = (double)mo.u[1];
                    if constexpr (D3) a.f_u[2 * nn + idx] = (double)mo.u[2];
                }
            } else {
                const double phi = (double)mo.phi;
                const double u2 = (double)mo.u[0] * (double)mo.u[0] +
                                  (double)mo.u[1] * (double)mo.u[1] +
                                  (double)mo.u[2] * (double)mo.u[2];
                acc.v[0] += phi;
                acc.v[1] += phi > 0.5 ? 1.0 : 0.0;
                acc.v[2] += phi;
                acc.v[3] = fmin(acc.v[3], phi);
                acc.v[4] = fmax(acc.v[4], phi);
                acc.v[5] = fmax(acc.v[5], u2);
                const bool bad = !isfinite(phi) || !isfinite(u2) || !((double)mo.rho > 0.0);
                acc.v[10] = fmax(acc.v[10], bad ? 1.0 : 0.0);
                if (a.has_centre) {
                    const double co[3] = {(double)x, (double)y, (double)z};
                    const int n[3] = {nx, ny, nz};
                    double r2 = 0.0;
                    for (int ax = 0; ax < PAIR::dim; ++ax) {
                        double d = co[ax] - a.centre[ax];
                        if (a.bc[ax] == 0) d -= n[ax] * rint(d / n[ax]);
                        r2 += d * d;
                    }
                    const double r = sqrt(r2);
                    if (r < a.r_in) { acc.v[6] += (double)mo.p; acc.v[7] += 1.0; }
                    if (r > a.r_out) { acc.v[8] += (double)mo.p; acc.v[9] += 1.0; }
                }
            }
        }
    };

    T hc[QH];
    T hq[MUF ? QH : 1];   // own h of plane z + 1 (Liang2014 fills two planes ahead)
    GS gr[QG];
    if constexpr (D3) {
        // ring of phi planes: plane zz lives in slot phi_slot(zz), filled ZL
        // planes ahead of the node plane. With 4 slots (ZL = 1): while a wave
        // fills plane z + 2 the slowest may still read planes z - 1 .. z + 1,
        // so one barrier per plane suffices. Liang2014 (ZL = 2, 5 slots, a
        // mu ring of 4): fill phi of z + 2, barrier, mu of z + 1 from phi
        // z .. z + 2, barrier, node update of z from phi and mu of z - 1 .. z + 1;
        // the fill of z + 3 then overwrites only phi of z - 2 and mu of z + 2
        // only mu of z - 2, which no wave still reads.
        for (int k = 0; k < 2 * ZL; ++k) {
            fill_plane(zs - ZL + k, phi_slot(zs - ZL + k));
            if (k == ZL) unroll<QH>([&](auto J) { constexpr int al = J; hc[al] = hn[al]; });
        }
        if constexpr (MUF) {
            unroll<QH>([&](auto J) { constexpr int al = J; hq[al] = hn[al]; });
            __syncthreads();
            fill_mu(zs - 1);
            fill_mu(zs);
        }
        for (int zl = zs; zl < ze; ++zl) {
            // the plane index is uniform; readfirstlane keeps the compiler from
            // treating it as per-lane after the divergent node branch (which
            // would move all plane and address arithmetic to 64-bit VALU)
            const int z = __builtin_amdgcn_readfirstlane(zl);
            for (int dy = 0; dy < 3; ++dy)
                for (int dx = 0; dx < 3; ++dx) lane_opaque(cl.off[dy][dx]);
            lane_opaque(ocr);
            for (int k = 0; k < NR; ++k) lane_opaque(rcr[k]);
            fill_plane(z + ZL, phi_slot(z + ZL));
            __syncthreads();
            if constexpr (MUF) {
                fill_mu(z + 1);
                __syncthreads();
            }
            if (active) {
                pull_g(z, gr);
                do_node(z, gr, hc, phi_slot(z - 1), phi_slot(z), phi_slot(z + 1));
            }
            if constexpr (MUF) {
                unroll<QH>([&](auto J) { constexpr int al = J; hc[al] = hq[al]; hq[al] = hn[al]; });
            } else {
                unroll<QH>([&](auto J) { constexpr int al = J; hc[al] = hn[al]; });
            }
        }
    } else {
        fill_plane(0, 0);
        __syncthreads();
        if constexpr (MUF) {
            fill_mu(0);
            __syncthreads();
        }
        if (active) {
            pull_g(0, gr);
            do_node(0, gr, hn, 0, 0, 0);
        }
    }
    if constexpr (MODE == MODE_DIAG) {
        __syncthreads();
        block_reduce_diag(acc, a.partials + (size_t)blockIdx.x * NDIAG);
    }
}

template <class PAIR, int MODEL, int PREC>
inline hipError_t step_mode(int mode, const KArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)(a.ntx * a.nty * a.ntz)), block(TILE_THREADS[a.tile]);
    const bool walls = a.wall_axis >= 0;
    switch (mode) {
        case MODE_STEP:
            if constexpr (PAIR::dim == 3) {
                if (a.tile == 1) {
                    if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 1, 1>), grid, block, 0, s, a);
                    else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 0, 1>), grid, block, 0, s, a);
                    break;
                }
                if (a.tile == 2) {
                    if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 1, 2>), grid, block, 0, s, a);
                    else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 0, 2>), grid, block, 0, s, a);
                    break;
                }
                if (a.tile == 3) {
                    if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 1, 3>), grid, block, 0, s, a);
                    else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 0, 3>), grid, block, 0, s, a);
                    break;
                }
                if (a.tile == 4) {
                    if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 1, 4>), grid, block, 0, s, a);
                    else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 0, 4>), grid, block, 0, s, a);
                    break;
                }
            }
            if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 1, 0>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_STEP, 0, 0>), grid, block, 0, s, a);
            break;
        case MODE_FIELDS:
            hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_FIELDS, 1, 0>), grid, block, 0, s, a);
            break;
        case MODE_RECORD:
            // float64 and float32 forms, tiles 64 x 4 and 128 x 2
            if constexpr (PREC <= 1) {
                if constexpr (PAIR::dim == 3) {
                    if (a.tile == 1) {
                        if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_RECORD, 1, 1>), grid, block, 0, s, a);
                        else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_RECORD, 0, 1>), grid, block, 0, s, a);
                        break;
                    }
                }
                if (a.tile != 0) return hipErrorInvalidValue;
                if (walls) hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_RECORD, 1, 0>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_RECORD, 0, 0>), grid, block, 0, s, a);
                break;
            }
            return hipErrorInvalidValue;
        default:
            hipLaunchKernelGGL((k_step<PAIR, MODEL, PREC, MODE_DIAG, 1, 0>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

// resident workgroups per compute unit of the 3-D step kernel with this tile
// (0 when the runtime cannot say)
template <class PAIR, int MODEL, int PREC, int WALLS>
inline int step_occupancy_walls(int tile) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const int bs = TILE_THREADS[tile];
    if constexpr (PAIR::dim == 3) {
        switch (tile) {
            case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<PAIR, MODEL, PREC, MODE_STEP, WALLS, 0>, bs, 0); break;
            case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<PAIR, MODEL, PREC, MODE_STEP, WALLS, 1>, bs, 0); break;
            case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<PAIR, MODEL, PREC, MODE_STEP, WALLS, 2>, bs, 0); break;
            case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<PAIR, MODEL, PREC, MODE_STEP, WALLS, 3>, bs, 0); break;
            case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<PAIR, MODEL, PREC, MODE_STEP, WALLS, 4>, bs, 0); break;
            default: break;
        }
    }
    return e == hipSuccess ? n : 0;
}

template <class PAIR, int MODEL>
inline int step_occupancy(int prec, int tile, int walls) {
    switch (prec) {
        case 0: return walls ? step_occupancy_walls<PAIR, MODEL, 0, 1>(tile) : step_occupancy_walls<PAIR, MODEL, 0, 0>(tile);
        case 1: return walls ? step_occupancy_walls<PAIR, MODEL, 1, 1>(tile) : step_occupancy_walls<PAIR, MODEL, 1, 0>(tile);
        case 2: return walls ? step_occupancy_walls<PAIR, MODEL, 2, 1>(tile) : step_occupancy_walls<PAIR, MODEL, 2, 0>(tile);
        default: return walls ? step_occupancy_walls<PAIR, MODEL, 3, 1>(tile) : step_occupancy_walls<PAIR, MODEL, 3, 0>(tile);
    }
}

template <class PAIR, int MODEL>
inline hipError_t step_prec(int prec, int mode, const KArgs& a, hipStream_t s) {
    switch (prec) {
        case 0: return step_mode<PAIR, MODEL, 0>(mode, a, s);
        case 1: return step_mode<PAIR, MODEL, 1>(mode, a, s);
        case 2: return step_mode<PAIR, MODEL, 2>(mode, a, s);
        default: return step_mode<PAIR, MODEL, 3>(mode, a, s);
    }
}

}  // namespace pfk
