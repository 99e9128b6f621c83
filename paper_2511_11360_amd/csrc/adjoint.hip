// Discrete adjoint of one time step of the fused step kernel, float64, on
// canonical arrays [q][z][y][x]: the conservative Allen-Cahn model (Sec.
// II.C.1 of the paper), and the CH (Sec. II.D.1), nonlocal / hybrid AC (Secs.
// II.C.3-4) and Liang2018 (Sec. II.C.2) variants.
//
// The forward step maps the post-streaming state X^n = (g, h) to X^{n+1}:
//   phi = sum h;  grad phi, lap phi from phi at x + c_i (periodic image or wall
//   mirror);  per node collision C(g, h, phi, grad phi, lap phi; sigma, M, W);
//   streaming (a permutation, bounce-back at walls plus a constant).
// Its adjoint maps lambda^{n+1} = dL/dX^{n+1} to lambda^n = dL/dX^n and adds
// dL/d(sigma, M, W) of the step:
//   pass 1  phi^n into the workspace;
//   pass 2  per node: lambda* (stream transpose, a gather), the reverse sweep
//           of C written out by hand (forward intermediates recomputed), giving
//           dL/dg (the new lambda_g), dL/dh through h directly, dL/dphi
//           directly, dL/dgrad phi, dL/dlap phi and the parameter terms
//           (block partials in float64);
//   pass 3  per node: transpose of the two stencils as a gather, added to every
//           h population (phi = sum h), plus the direct term of h (the h stream
//           transpose of lambda_h^{n+1} times 1 - 1/tau_phi).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "lattice.h"
#include "pflbm.h"

namespace pfk {

// Device scratch of pflbm_adjoint_step_noalloc, for callers that cannot
// allocate: phi, the five per-node adjoint values and the per-workgroup
// parameter partials of one adjoint step, for boxes of up to 128^3 nodes.
// Every GPU the library runs on holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that device (adjoint_scratch below).
static __device__ __align__(256) char scratch[PFLBM_ADJOINT_SCRATCH_BYTES];

hipError_t adjoint_scratch(int device, void** out) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void* ptrs[MAXDEV] = {};
    if (device < 0 || device >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptrs[device] = p;
    }
    *out = ptrs[device];
    return hipSuccess;
}

namespace {

struct Node {
    int x, y, z;
};

// node coordinates of linear index n (boxes hold fewer than 2^31 nodes, so
// 32-bit division suffices)
template <class A>
__device__ __forceinline__ Node node_of(long long n, const A& a) {
    const int m = (int)n;
    const int q = m / a.nx;
    Node d;
    d.x = m - q * a.nx;
    d.y = q % a.ny;
    d.z = q / a.ny;
    return d;
}

// workgroup index in row order: consecutive hardware indices go round-robin
// to the eight XCDs, so the first 8 * (nb / 8) are regrouped so that each XCD
// takes a contiguous run of rows (the y neighbours of a row then sit in the
// same L2); the remainder keeps its index
__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, per = gridDim.x / 8;
    return b < 8 * per ? (b % 8) * per + b / 8 : b;
}

// neighbours of one node, formed once: along each axis the coordinates v - 1,
// v, v + 1 (periodic image, or clamped to the wall layer with the "beyond"
// flag set when the node lies beyond a wall); the linear index of x + c is a
// plane offset plus a row offset plus a column
struct Nbr {
    long long zo[3];
    int yo[3], xo[3];
    bool bnd[3][3];

    template <class A>
    __device__ __forceinline__ Nbr(const A& a, Node p) {
        const int v[3] = {p.x, p.y, p.z};
        const int n3[3] = {a.nx, a.ny, a.nz};
        int o[3][3];
        for (int d = 0; d < 3; ++d)
            for (int k = 0; k < 3; ++k) {
                const int w = v[d] - 1 + k, n = n3[d];
                const bool out = w < 0 || w >= n;
                bnd[d][k] = out && a.bc[d] != 0;
                o[d][k] = !out ? w : (a.bc[d] == 0 ? (w < 0 ? w + n : w - n) : (w < 0 ? 0 : n - 1));
            }
        for (int k = 0; k < 3; ++k) {
            xo[k] = o[0][k];
            yo[k] = o[1][k] * a.nx;
            zo[k] = (long long)o[2][k] * a.nx * a.ny;
        }
    }
    // x + c, wrapped, or clamped onto the wall layer
    __device__ __forceinline__ long long index(int cx, int cy, int cz) const {
        return zo[cz + 1] + yo[cy + 1] + xo[cx + 1];
    }
    // whether x + c lies beyond a wall
    __device__ __forceinline__ bool beyond(int cx, int cy, int cz) const {
        return (cx != 0 && bnd[0][cx + 1]) || (cy != 0 && bnd[1][cy + 1]) || (cz != 0 && bnd[2][cz + 1]);
    }
};

// stress row k of the two-rate collision evaluated at velocity i: 3 c_x^2 - c^2,
// c_y^2 - c_z^2, c_x c_y, c_y c_z, c_x c_z (2-D: c_x^2 - c_y^2, 0, c_x c_y, 0, 0)
template <class GL, bool D3>
__host__ __device__ constexpr int stress_row(int k, int i) {
    const int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
    if (k == 0) return D3 ? 3 * cx * cx - (cx * cx + cy * cy + cz * cz) : cx * cx - cy * cy;
    if (k == 1) return D3 ? cy * cy - cz * cz : 0;
    if (k == 2) return cx * cy;
    if (k == 3) return cy * cz;
    return cx * cz;
}
// its squared norm over the velocity set (the projector's denominator; 36,
// 12, 4 on D3Q19 and 36, 12, 12 on D3Q27 for the rows of each kind)
template <class GL, bool D3>
__host__ __device__ constexpr double stress_norm(int k) {
    int s = 0;
    for (int i = 0; i < GL::Q; ++i) s += stress_row<GL, D3>(k, i) * stress_row<GL, D3>(k, i);
    return s > 0 ? (double)s : 1.0;
}

// the rows' coefficients of the two-rate projector for the traceless
// stress Pi (each row's sum over the populations divided by its squared
// norm), and their transpose (added into b_Pi, upper triangle)
template <class GL, bool D3, class R>
__device__ __forceinline__ void stress_coeffs(const R (&Pi)[3][3], R (&A)[5]) {
    constexpr R N0 = stress_norm<GL, D3>(0), N1 = stress_norm<GL, D3>(1), N2 = stress_norm<GL, D3>(2),
                N3 = stress_norm<GL, D3>(3), N4 = stress_norm<GL, D3>(4);
    if constexpr (D3) {
        A[0] = (R(2) * Pi[0][0] - Pi[1][1] - Pi[2][2]) / N0;
        A[1] = (Pi[1][1] - Pi[2][2]) / N1;
        A[2] = Pi[0][1] / N2;
        A[3] = Pi[1][2] / N3;
        A[4] = Pi[0][2] / N4;
    } else {
        A[0] = (Pi[0][0] - Pi[1][1]) / N0;
        A[1] = R(0);
        A[2] = Pi[0][1] / N2;
        A[3] = R(0);
        A[4] = R(0);
    }
}
template <class GL, bool D3, class R>
__device__ __forceinline__ void stress_coeffs_T(const R (&b_A)[5], R (&b_Pi)[3][3]) {
    constexpr R N0 = stress_norm<GL, D3>(0), N1 = stress_norm<GL, D3>(1), N2 = stress_norm<GL, D3>(2),
                N3 = stress_norm<GL, D3>(3), N4 = stress_norm<GL, D3>(4);
    if constexpr (D3) {
        b_Pi[0][0] += R(2) * b_A[0] / N0;
        b_Pi[1][1] += -b_A[0] / N0 + b_A[1] / N1;
        b_Pi[2][2] += -b_A[0] / N0 - b_A[1] / N1;
        b_Pi[0][1] += b_A[2] / N2;
        b_Pi[1][2] += b_A[3] / N3;
        b_Pi[0][2] += b_A[4] / N4;
    } else {
        b_Pi[0][0] += b_A[0] / N0;
        b_Pi[1][1] += -b_A[0] / N0;
        b_Pi[0][1] += b_A[2] / N2;
    }
}

// moments of the hydrodynamic populations: sum g, sum c g, sum c c g; and
// the transpose, added into b_g (b_m2 upper triangle)
template <class GL, class R>
__device__ __forceinline__ void moments(const R (&g)[GL::Q], R& ps, R (&j)[3], R (&m2)[3][3]) {
    ps = R(0);
    for (int k = 0; k < 3; ++k) {
        j[k] = R(0);
        for (int l = 0; l < 3; ++l) m2[k][l] = R(0);
    }
    unroll<GL::Q>([&](auto I) {
        constexpr int i = I;
        ps += g[i];
        for (int k = 0; k < 3; ++k) {
            j[k] += GL::c(i, k) * g[i];
            for (int l = 0; l < 3; ++l) m2[k][l] += GL::c(i, k) * GL::c(i, l) * g[i];
        }
    });
}
template <class GL, class R>
__device__ __forceinline__ void moments_T(R b_ps, const R (&b_j)[3], const R (&b_m2)[3][3], R (&b_g)[GL::Q]) {
    for (int i = 0; i < GL::Q; ++i) {
        R b = b_ps;
        for (int k = 0; k < 3; ++k) {
            b += GL::c(i, k) * b_j[k];
            for (int l = k; l < 3; ++l) b += GL::c(i, k) * GL::c(i, l) * b_m2[k][l];
        }
        b_g[i] += b;
    }
}

// dL/dphi through nu(phi) (linear mu over rho, or linear nu), irho = 1 /
// rho(phi) and rho = rhoL + phi dRho, from their adjoints
template <class R>
__device__ __forceinline__ R phys_T(const PhysT<R>& ph, R irho, R numu, R b_nu, R b_irho, R b_rho) {
    R b_phi = R(0);
    if (ph.visc_mu) {
        b_phi += ph.dMu * irho * b_nu;
        b_irho += numu * b_nu;
    } else {
        b_phi += ph.dNu * b_nu;
    }
    b_rho += -irho * irho * b_irho;
    return b_phi + ph.dRho * b_rho;
}

// the physical parameters in the arithmetic type of a kernel (float64: the
// kernel argument itself, read where used)
template <class R>
__device__ __forceinline__ decltype(auto) phys_as(const Phys& p) {
    if constexpr (sizeof(R) == sizeof(double)) return (p);
    else return to_float(p);
}

// 256-thread fixed-order block sums of K values per thread into
// part[wg * STRIDE + k] (ADD: added to what is there)
template <int K, int STRIDE, bool ADD = false>
__device__ __forceinline__ void block_sums(const double (&v)[K], double* part, int wg) {
    __shared__ double red[K][256];
    for (int k = 0; k < K; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) {
            if constexpr (ADD) part[(size_t)wg * STRIDE + k] += red[k][0];
            else part[(size_t)wg * STRIDE + k] = red[k][0];
        }
}

}  // namespace

template <class R>
__global__ __launch_bounds__(256) void k_adj_phi(const AdjArgsT<R> a) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    // summed in float64 also for the float32 adjoint: where phi is near 1
    // and its gradient small (inside a droplet), the interface normal's
    // adjoint scales with 1 / |grad phi|, and float32 differences of phi
    // would carry absolute errors of one float32 ulp of 1 into it
    double s = a.fh[n];
    for (int al = 1; al < a.qh; ++al) s += a.fh[(size_t)al * nn + n];
    a.phi[n] = s;
}

// pass 2: local reverse sweep of the collision. MODEL 0: conservative AC
// (Eqs. fakhari_geq, fakhari_G_modified); MODEL 1: the Cahn-Hilliard phase
// field (Eqs. liang2_geq, liang2_G with the backward-Euler d(phi u)/dt, whose
// (phi u) of the previous step is part of the state); MODEL 2: the nonlocal
// AC (Eqs. Chai_geq, Hu_G; phi here is the corrected phi* of the phase-field
// pass, the nonlocal source R is formed from sum h of the node)
template <class PAIR, int MODEL, class R = double>
__global__ __launch_bounds__(256, 2) void k_adj_local(const AdjArgsT<R> a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    constexpr int Q = GL::Q, QH = HL::Q;
    constexpr bool D3 = PAIR::dim == 3;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double th[3] = {R(0.0), R(0.0), R(0.0)};   // d sigma, d M, d W of this node
    if (n < nn) {
        const Node p = node_of(n, a);
        const auto& ph = phys_as<R>(a.ph);
        R g[Q], h[QH];
        double phin[Q];
        for (int i = 0; i < Q; ++i) g[i] = a.fg[(size_t)i * nn + n];
        for (int al = 0; al < QH; ++al) h[al] = a.fh[(size_t)al * nn + n];
        const Nbr nb(a, p);
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            phin[i] = a.phi[nb.index(GL::c(i, 0), GL::c(i, 1), GL::c(i, 2))];
        });
        // ---------------- forward intermediates (as in the step kernel); the
        // stencils and phi (1 - phi) are formed in float64 from the float64
        // phi and rounded once (no cancellation left for the float32 form)
        const R phi = R(phin[0]);
        R gr[3], lap;
        {
            double grd[3] = {0.0, 0.0, 0.0}, lapd = 0.0;
            unroll<Q>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    for (int k = 0; k < 3; ++k) grd[k] += 3.0 * GL::w(i) * GL::c(i, k) * phin[i];
                    lapd += 6.0 * GL::w(i) * (phin[i] - phin[0]);
                }
            });
            for (int k = 0; k < 3; ++k) gr[k] = R(grd[k]);
            lap = R(lapd);
        }
        const R dR = ph.dRho;
        const R rho = ph.rhoL + phi * dR;
        const R irho = R(1.0) / rho;
        const R numu = ph.muL + phi * ph.dMu;
        const R nu = ph.visc_mu ? numu * irho : ph.nuL + phi * ph.dNu;
        const R tau = R(3.0) * nu + R(0.5);
        const R itau = R(1.0) / tau;
        const R cub = R(phin[0] * (phin[0] - 1.0) * (phin[0] - 0.5));
        const R mu = ph.beta4 * cub - ph.kappa * lap;
        R ps, j[3], m2[3][3];
        moments<GL>(g, ps, j, m2);
        const R sg = mu - ps * dR / R(3.0);
        R F0[3], us[3], S[3][3], F[3], u[3];
        for (int k = 0; k < 3; ++k) F0[k] = sg * gr[k] + rho * ph.body[k] + ph.force[k];
        for (int k = 0; k < 3; ++k) us[k] = j[k] + F0[k] * R(0.5) * irho;
        const R s3 = ps / R(3.0);
        const R sfac = -R(3.0) * itau;
        const int dmax = D3 ? 3 : 2;
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                S[k][l] = (k < dmax && l < dmax)
                              ? sfac * (m2[k][l] - (k == l ? s3 : R(0.0)) - us[k] * us[l]) : R(0.0);
        const R nr = nu * dR;
        R Sg[3];
        for (int k = 0; k < 3; ++k) Sg[k] = S[k][0] * gr[0] + S[k][1] * gr[1] + S[k][2] * gr[2];
        for (int k = 0; k < 3; ++k) F[k] = F0[k] + nr * Sg[k];
        for (int k = 0; k < 3; ++k) u[k] = j[k] + F[k] * R(0.5) * irho;
        const R usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const R so = ph.s_o;
        const R dS = itau - so;
        const R ffac = (R(1.0) - R(0.5) * so) * R(3.0) * irho;
        const R aeq = ps - R(1.5) * usq;
        R Pi[3][3];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                Pi[k][l] = m2[k][l] - (k == l ? s3 : R(0.0)) - u[k] * u[l];
        // stress-projection coefficients (linear in Pi), each row's sum over
        // the populations divided by its squared norm
        R A[5];
        stress_coeffs<GL, D3>(Pi, A);
        auto qrow = [&](int i, R* q) {   // stress rows evaluated at c_i
            for (int k = 0; k < 5; ++k) q[k] = stress_row<GL, D3>(k, i);
        };
        const R gg = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        const R sn = gg + ph.eps2;
        const R rn = sn > R(0.0) ? R(1.0) / sqrt(sn) : R(0.0);   // guarded normal at eps = 0
        const R pp = R(phin[0] * (1.0 - phin[0]));
        const R coef = ph.anti * pp * rn;
        const R itp = ph.inv_tau_phi, gfp = ph.g_fac_phi;
        // CH: (phi u) of this step and of the previous one (state)
        R puc[3] = {R(0.0), R(0.0), R(0.0)}, pup[3] = {R(0.0), R(0.0), R(0.0)};
        if constexpr (MODEL == 1) {
            for (int k = 0; k < 3; ++k) {
                puc[k] = phi * u[k];
                pup[k] = a.fpu[(size_t)k * nn + n];
            }
        }

        // ---------------- reverse sweep
        // lambda* : adjoint of the post-collision populations (stream transpose),
        // gathered here, where the sweep first needs it;
        // beyond a wall, the bounce-back slot opp(i) of the node itself
        R lg[Q], lh[QH];
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)GL::opp(i) * nn + n
                                                    : (size_t)i * nn + nb.index(cx, cy, cz);
            lg[i] = a.lg[e];
        });
        unroll<QH>([&](auto J) {
            constexpr int al = J;
            constexpr int cx = HL::c(al, 0), cy = HL::c(al, 1), cz = HL::c(al, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)HL::opp(al) * nn + n
                                                    : (size_t)al * nn + nb.index(cx, cy, cz);
            lh[al] = a.lh[e];
        });
        R b_g[Q];
        R b_phi = R(0.0), b_gr[3] = {R(0.0), R(0.0), R(0.0)}, b_lap = R(0.0);
        R b_u[3] = {R(0.0), R(0.0), R(0.0)}, b_F[3] = {R(0.0), R(0.0), R(0.0)};
        R b_ps = R(0.0), b_irho = R(0.0), b_itau = R(0.0), b_usq = R(0.0), b_aeq = R(0.0);
        R b_coef = R(0.0), b_anti = R(0.0), b_itp = R(0.0), b_gfp = R(0.0);
        R b_Pi[3][3] = {{R(0.0)}};
        R b_muh = R(0.0);   // CH: mu_phi through h_eq
        R b_R = R(0.0);     // nonlocal: the source R through G

        if constexpr (MODEL == 1) {
            // h*_a = (1 - itp) h_a + itp heq_a + gfp G_a with
            // heq_0 = phi + (w_0 - 1) eta mu, heq_a = w_a eta mu + 3 w_a e_a . (phi u),
            // G_a = 3 w_a e_a . ((phi u) - (phi u)_prev); (phi u) is also stored
            // for the next step, whose adjoint lambda_pu^{n+1} arrives at the node
            R b_puc[3], b_pup[3] = {R(0.0), R(0.0), R(0.0)};
            for (int k = 0; k < 3; ++k) b_puc[k] = a.lpu[(size_t)k * nn + n];
            unroll<QH>([&](auto J) {
                constexpr int al = J;
                constexpr R w = R(HL::w(al));
                constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
                const R lb = lh[al];
                const R bheq = itp * lb;
                R heq, G = R(0.0);
                if constexpr (al == 0) {
                    heq = phi + (w - R(1.0)) * ph.eta * mu;
                    b_phi += bheq;
                    b_muh += (w - R(1.0)) * ph.eta * bheq;
                } else {
                    const R ep = ex * puc[0] + ey * puc[1] + ez * puc[2];
                    const R eq = ex * pup[0] + ey * pup[1] + ez * pup[2];
                    heq = w * ph.eta * mu + R(3.0) * w * ep;
                    G = R(3.0) * w * (ep - eq);
                    b_muh += w * ph.eta * bheq;
                    const R t = R(3.0) * w * (bheq + gfp * lb);
                    const R tp = R(3.0) * w * gfp * lb;
                    b_puc[0] += ex * t;
                    b_puc[1] += ey * t;
                    b_puc[2] += ez * t;
                    b_pup[0] -= ex * tp;
                    b_pup[1] -= ey * tp;
                    b_pup[2] -= ez * tp;
                }
                // heq_0 - h_0 = (phi - h_0) + (w_0 - 1) eta mu, phi - h_0 formed
                // in float64 (h_0 carries nearly all of phi)
                if constexpr (al == 0)
                    b_itp += (R(phin[0] - (double)h[0]) + (w - R(1.0)) * ph.eta * mu) * lb;
                else
                    b_itp += (heq - h[al]) * lb;
                b_gfp += G * lb;
            });
            // (phi u) = phi u
            for (int k = 0; k < 3; ++k) {
                b_phi += u[k] * b_puc[k];
                b_u[k] += phi * b_puc[k];
                a.opu[(size_t)k * nn + n] = b_pup[k];
            }
        } else if constexpr (MODEL == 2) {
            // h*_a = (1 - itp) h_a + itp heq_a + gfp G_a with heq_a = w_a phi
            // (1 + 3 e_a . u), G_a = lam w_a coef (e_a . gr) + (1 - lam) w_a R,
            // R = M (gamma phi_s (1 - phi_s) - (32 / W^2) phi_s (phi_s - 1)
            // (phi_s - 1/2)) at phi_s = sum h (summed in the phi pass's order)
            R hs = h[0];
            for (int al = 1; al < QH; ++al) hs += h[al];
            const R gam = a.nls[0];
            const R Rs = ph.mob * (gam * hs * (R(1.0) - hs) - ph.w32 * (hs - R(1.0)) * hs * (hs - R(0.5)));
            const R lam = ph.lam;
            for (int al = 0; al < QH; ++al) {
                const R w = R(HL::w(al));
                const R eu = HL::c(al, 0) * u[0] + HL::c(al, 1) * u[1] + HL::c(al, 2) * u[2];
                const R eg = HL::c(al, 0) * gr[0] + HL::c(al, 1) * gr[1] + HL::c(al, 2) * gr[2];
                const R heq = w * phi * (R(1.0) + R(3.0) * eu);
                const R lb = lh[al];
                b_itp += (heq - h[al]) * lb;
                b_gfp += (lam * w * coef * eg + (R(1.0) - lam) * w * Rs) * lb;
                b_coef += gfp * lam * w * eg * lb;
                for (int k = 0; k < 3; ++k) b_gr[k] += gfp * lam * w * coef * HL::c(al, k) * lb;
                b_R += gfp * (R(1.0) - lam) * w * lb;
                const R bheq = itp * lb;
                b_phi += bheq * w * (R(1.0) + R(3.0) * eu);
                for (int k = 0; k < 3; ++k) b_u[k] += bheq * w * phi * R(3.0) * HL::c(al, k);
            }
            b_anti += b_coef * pp * rn;
            b_phi += b_coef * ph.anti * (R(1.0) - R(2.0) * phi) * rn;
            const R b_rn = b_coef * ph.anti * pp;
            const R b_gg = -R(0.5) * rn * rn * rn * b_rn;
            for (int k = 0; k < 3; ++k) b_gr[k] += R(2.0) * gr[k] * b_gg;
        } else {
        // h*_a = (1 - itp) h_a + itp heq_a + gfp w_a coef (e_a . gr); the
        // non-equilibrium heq_a - h_a (small against h_a) as (w_a phi - h_a),
        // formed in float64, plus w_a phi (base - 1)
        for (int al = 0; al < QH; ++al) {
            const R w = R(HL::w(al));
            const R eu = HL::c(al, 0) * u[0] + HL::c(al, 1) * u[1] + HL::c(al, 2) * u[2];
            const R eg = HL::c(al, 0) * gr[0] + HL::c(al, 1) * gr[1] + HL::c(al, 2) * gr[2];
            const R bm1 = R(3.0) * eu + R(4.5) * eu * eu - R(1.5) * usq;
            const R base = R(1.0) + bm1;
            const R lb = lh[al];
            b_itp += (R(HL::w(al) * phin[0] - (double)h[al]) + w * phi * bm1) * lb;
            b_gfp += w * coef * eg * lb;
            b_coef += gfp * w * eg * lb;
            for (int k = 0; k < 3; ++k) b_gr[k] += gfp * w * coef * HL::c(al, k) * lb;
            const R bheq = itp * lb;
            b_phi += bheq * w * base;
            for (int k = 0; k < 3; ++k)
                b_u[k] += bheq * w * phi * (R(3.0) * HL::c(al, k) + R(9.0) * eu * HL::c(al, k));
            b_usq += -R(1.5) * bheq * w * phi;
        }
        // coef = anti phi (1 - phi) (gg + eps^2)^(-1/2)
        b_anti += b_coef * pp * rn;
        b_phi += b_coef * ph.anti * (R(1.0) - R(2.0) * phi) * rn;
        {
            const R b_rn = b_coef * ph.anti * pp;
            const R b_gg = -R(0.5) * rn * rn * rn * b_rn;
            for (int k = 0; k < 3; ++k) b_gr[k] += R(2.0) * gr[k] * b_gg;
        }
        }
        // g*_i = (1 - so) g_i + so geq_i - dS P_i + ffac w_i (c_i . F)
        R b_A[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
        R b_dS = R(0.0), b_ffac = R(0.0);
        for (int i = 0; i < Q; ++i) {
            const R w = R(GL::w(i));
            const R cu = GL::c(i, 0) * u[0] + GL::c(i, 1) * u[1] + GL::c(i, 2) * u[2];
            const R cf = GL::c(i, 0) * F[0] + GL::c(i, 1) * F[1] + GL::c(i, 2) * F[2];
            R q[5];
            qrow(i, q);
            R P = R(0.0);
            for (int k = 0; k < 5; ++k) P += q[k] * A[k];
            const R lb = lg[i];
            b_g[i] = (R(1.0) - so) * lb;
            const R bgeq = so * lb;
            b_aeq += w * bgeq;
            for (int k = 0; k < 3; ++k) b_u[k] += w * bgeq * (R(3.0) * GL::c(i, k) + R(9.0) * cu * GL::c(i, k));
            for (int k = 0; k < 5; ++k) b_A[k] += -dS * q[k] * lb;
            b_dS += -P * lb;
            b_ffac += w * cf * lb;
            for (int k = 0; k < 3; ++k) b_F[k] += ffac * w * GL::c(i, k) * lb;
        }
        // A (linear in Pi)
        stress_coeffs_T<GL, D3>(b_A, b_Pi);
        // Pi_kl = m2_kl - delta s3 - u_k u_l (only k <= l entries carry adjoints)
        R b_m2[3][3] = {{R(0.0)}}, b_s3 = R(0.0);
        for (int k = 0; k < 3; ++k)
            for (int l = k; l < 3; ++l) {
                const R b = b_Pi[k][l];
                b_m2[k][l] += b;
                if (k == l) {
                    b_s3 -= b;
                    b_u[k] -= R(2.0) * u[k] * b;
                } else {
                    b_u[k] -= u[l] * b;
                    b_u[l] -= u[k] * b;
                }
            }
        // aeq = ps - 1.5 usq ; usq = u.u ; dS = itau - so ; ffac = (1 - so/2) 3 irho
        b_ps += b_aeq;
        b_usq += -R(1.5) * b_aeq;
        for (int k = 0; k < 3; ++k) b_u[k] += R(2.0) * u[k] * b_usq;
        b_itau += b_dS;
        b_irho += (R(1.0) - R(0.5) * so) * R(3.0) * b_ffac;
        // u = j + F irho / 2
        R b_j[3];
        for (int k = 0; k < 3; ++k) {
            b_j[k] = b_u[k];
            b_F[k] += R(0.5) * irho * b_u[k];
            b_irho += R(0.5) * F[k] * b_u[k];
        }
        // F = F0 + nr S gr
        R b_F0[3], b_S[3][3] = {{R(0.0)}}, b_nr = R(0.0);
        for (int k = 0; k < 3; ++k) {
            b_F0[k] = b_F[k];
            b_nr += b_F[k] * Sg[k];
            for (int l = 0; l < 3; ++l) {
                b_S[k][l] += nr * b_F[k] * gr[l];
                b_gr[l] += nr * S[k][l] * b_F[k];
            }
        }
        R b_nu = b_nr * dR;
        // S_kl = sfac (m2_kl - delta s3 - us_k us_l)  (full symmetric 3 x 3)
        R b_us[3] = {R(0.0), R(0.0), R(0.0)}, b_sfac = R(0.0);
        for (int k = 0; k < dmax; ++k)
            for (int l = 0; l < dmax; ++l) {
                const R b = b_S[k][l];
                b_sfac += b * (m2[k][l] - (k == l ? s3 : R(0.0)) - us[k] * us[l]);
                const R bs = sfac * b;
                if (k <= l) b_m2[k][l] += bs;
                else b_m2[l][k] += bs;
                if (k == l) b_s3 -= bs;
                b_us[k] -= bs * us[l];
                b_us[l] -= bs * us[k];
            }
        b_itau += -R(3.0) * b_sfac;
        b_ps += b_s3 / R(3.0);
        // us = j + F0 irho / 2
        for (int k = 0; k < 3; ++k) {
            b_j[k] += b_us[k];
            b_F0[k] += R(0.5) * irho * b_us[k];
            b_irho += R(0.5) * F0[k] * b_us[k];
        }
        // F0 = sg gr + rho body + force
        R b_sg = R(0.0), b_rho = R(0.0);
        for (int k = 0; k < 3; ++k) {
            b_sg += b_F0[k] * gr[k];
            b_gr[k] += sg * b_F0[k];
            b_rho += ph.body[k] * b_F0[k];
        }
        // sg = mu - ps dR / 3
        const R b_mu = b_sg + b_muh;
        b_ps += -b_sg * dR / R(3.0);
        // moments
        moments_T<GL>(b_ps, b_j, b_m2, b_g);
        // mu = beta4 phi (phi - 1)(phi - 1/2) - kappa lap
        const R b_beta4 = b_mu * cub;
        const R b_kappa = -b_mu * lap;
        b_lap += -ph.kappa * b_mu;
        b_phi += b_mu * ph.beta4 * (R(3.0) * phi * phi - R(3.0) * phi + R(0.5));
        // itau = 1 / tau, tau = 3 nu + 1/2; nu, irho = 1 / rho, rho = rhoL + phi dR
        b_nu += R(3.0) * (-itau * itau * b_itau);
        b_phi += phys_T(ph, irho, numu, b_nu, b_irho, b_rho);

        // parameters: beta4 = 48 sigma / W, kappa = 1.5 sigma W, anti = 4 / W,
        // itp = 1 / (3 M + 1/2), gfp = 1 - itp / 2 (the nonlocal source's M and
        // W terms are formed with its total adjoint, after the stencil pass)
        const R sigma = R(a.sigma), W = R(a.W);
        th[0] = b_beta4 * R(48.0) / W + b_kappa * R(1.5) * W;
        const R b_itp_tot = b_itp - R(0.5) * b_gfp;
        th[1] = -(MODEL == 1 ? R(3.0) / ph.eta : R(3.0)) * itp * itp * b_itp_tot;   // tau_phi = 3 M (/ eta) + 1/2
        th[2] = -b_beta4 * R(48.0) * sigma / (W * W) + b_kappa * R(1.5) * sigma - b_anti * R(4.0) / (W * W);

        for (int i = 0; i < Q; ++i) a.og[(size_t)i * nn + n] = b_g[i];
        // the direct h adjoint (1 - itp) lambda*_h is formed by the stencil pass
        a.work[n] = b_phi;
        a.work[nn + n] = b_gr[0];
        a.work[2 * nn + n] = b_gr[1];
        a.work[3 * nn + n] = b_gr[2];
        a.work[4 * nn + n] = b_lap;
        if constexpr (MODEL == 2) a.work[5 * nn + n] = b_R;
    }
    // block sums of the parameter adjoints, fixed order (written out rather
    // than through block_sums: with the helper the compiler spills 68 bytes
    // per lane in this sweep, with this form 20)
    __shared__ double red[3][256];
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = th[k];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) a.partials[(size_t)wg * 3 + k] = red[k][0];
}

// pass 2 for Liang2018 (Sec. II.C): its conservative-form hydrodynamics,
// f_eq of Eq. liang_feq, forcing of Eq. liang_F_final (F = F_s + F_b, with a
// stress part), rho u = sum e f + F / 2, p of Eq. liang_p_update, and the
// phase field of Eqs. liang_geq, liang_G_final (backward-Euler d(phi u)/dt:
// (phi u) of the previous step is part of the state). Same outputs as the
// other sweeps: dL/dg, dL/dphi, dL/dgrad phi, dL/dlap phi, dL/d(phi u)_prev
// and the parameter partials.
template <class PAIR>
__global__ __launch_bounds__(256, 2) void k_adj_local_l18(const AdjArgs a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    constexpr int Q = GL::Q, QH = HL::Q;
    constexpr bool D3 = PAIR::dim == 3;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double th[3] = {0.0, 0.0, 0.0};
    if (n < nn) {
        const Node p = node_of(n, a);
        const Phys& ph = a.ph;
        double g[Q], h[QH], phin[Q];
        for (int i = 0; i < Q; ++i) g[i] = a.fg[(size_t)i * nn + n];
        for (int al = 0; al < QH; ++al) h[al] = a.fh[(size_t)al * nn + n];
        const Nbr nb(a, p);
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            phin[i] = a.phi[nb.index(GL::c(i, 0), GL::c(i, 1), GL::c(i, 2))];
        });
        // ---------------- forward intermediates (as in the step kernel)
        const double phi = phin[0];
        double gr[3] = {0.0, 0.0, 0.0}, lap = 0.0;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                for (int k = 0; k < 3; ++k) gr[k] += 3.0 * GL::w(i) * GL::c(i, k) * phin[i];
                lap += 6.0 * GL::w(i) * (phin[i] - phi);
            }
        });
        const double dR = ph.dRho;
        const double rho = ph.rhoL + phi * dR;
        const double irho = 1.0 / rho;
        const double numu = ph.muL + phi * ph.dMu;
        const double nu = ph.visc_mu ? numu * irho : ph.nuL + phi * ph.dNu;
        const double itau = 1.0 / (3.0 * nu + 0.5);
        const double cub = phi * (phi - 1.0) * (phi - 0.5);
        const double mu = ph.beta4 * cub - ph.kappa * lap;
        double ps, j[3], m2[3][3];
        moments<GL>(g, ps, j, m2);
        double F[3], u[3], grho[3], jF[3];
        for (int k = 0; k < 3; ++k) {
            F[k] = mu * gr[k] + rho * ph.body[k] + ph.force[k];
            jF[k] = j[k] + 0.5 * F[k];
            u[k] = jF[k] * irho;
            grho[k] = dR * gr[k];
        }
        const double udr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
        const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        constexpr double w0 = GL::w(0);
        constexpr double cp = 1.0 / (3.0 * (1.0 - w0));
        const double pres = cp * ((ps - g[0]) + 0.5 * udr - 1.5 * rho * w0 * usq);
        const double so = ph.s_o;
        const double dS = itau - so;
        const double fh = 1.0 - 0.5 * so;
        const double p3 = 3.0 * pres;
        const double kin0 = -1.5 * rho * usq;
        double Pi[3][3];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                Pi[k][l] = m2[k][l] - rho * u[k] * u[l] + (1.0 / 6.0) * (u[k] * grho[l] + u[l] * grho[k]);
        double A[5];
        stress_coeffs<GL, D3>(Pi, A);
        const double gg = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        const double sn = gg + ph.eps2;
        const double rn = sn > 0.0 ? 1.0 / sqrt(sn) : 0.0;
        const double pp = phi * (1.0 - phi);
        const double coef = ph.anti * pp * rn;
        const double itp = ph.inv_tau_phi, gfp = ph.g_fac_phi;
        double pu[3], dpu[3];
        for (int k = 0; k < 3; ++k) {
            pu[k] = phi * u[k];
            dpu[k] = pu[k] - a.fpu[(size_t)k * nn + n];
        }

        // ---------------- reverse sweep; lambda* gathered through the stream transpose
        double lg[Q], lh[QH];
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)GL::opp(i) * nn + n
                                                    : (size_t)i * nn + nb.index(cx, cy, cz);
            lg[i] = a.lg[e];
        });
        unroll<QH>([&](auto J) {
            constexpr int al = J;
            constexpr int cx = HL::c(al, 0), cy = HL::c(al, 1), cz = HL::c(al, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)HL::opp(al) * nn + n
                                                    : (size_t)al * nn + nb.index(cx, cy, cz);
            lh[al] = a.lh[e];
        });
        double b_phi = 0.0, b_gr[3] = {0.0, 0.0, 0.0}, b_u[3] = {0.0, 0.0, 0.0};
        double b_itp = 0.0, b_gfp = 0.0, b_coef = 0.0;
        // h*_a = (1 - itp) h_a + itp w phi (1 + 3 e.u) + gfp w e.(3 dpu + coef gr)
        double b_pu[3], b_dpu[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3; ++k) b_pu[k] = a.lpu[(size_t)k * nn + n];   // (phi u) stored for the next step
        for (int al = 0; al < QH; ++al) {
            const double w = HL::w(al);
            const double ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
            const double eu = ex * u[0] + ey * u[1] + ez * u[2];
            const double eg = ex * gr[0] + ey * gr[1] + ez * gr[2];
            const double ed = ex * dpu[0] + ey * dpu[1] + ez * dpu[2];
            const double heq = w * phi * (1.0 + 3.0 * eu);
            const double G = w * (3.0 * ed + coef * eg);
            const double lb = lh[al];
            b_itp += (heq - h[al]) * lb;
            b_gfp += G * lb;
            const double bheq = itp * lb, bG = gfp * lb;
            b_phi += bheq * w * (1.0 + 3.0 * eu);
            b_u[0] += 3.0 * bheq * w * phi * ex;
            b_u[1] += 3.0 * bheq * w * phi * ey;
            b_u[2] += 3.0 * bheq * w * phi * ez;
            b_dpu[0] += 3.0 * bG * w * ex;
            b_dpu[1] += 3.0 * bG * w * ey;
            b_dpu[2] += 3.0 * bG * w * ez;
            b_coef += bG * w * eg;
            b_gr[0] += bG * w * coef * ex;
            b_gr[1] += bG * w * coef * ey;
            b_gr[2] += bG * w * coef * ez;
        }
        // dpu = pu - pu_prev, pu = phi u
        for (int k = 0; k < 3; ++k) {
            b_pu[k] += b_dpu[k];
            a.opu[(size_t)k * nn + n] = -b_dpu[k];
            b_phi += u[k] * b_pu[k];
            b_u[k] += phi * b_pu[k];
        }
        // coef = anti phi (1 - phi) (gg + eps^2)^(-1/2)
        const double b_anti = b_coef * pp * rn;
        b_phi += b_coef * ph.anti * (1.0 - 2.0 * phi) * rn;
        {
            const double b_gg = -0.5 * rn * rn * rn * b_coef * ph.anti * pp;
            for (int k = 0; k < 3; ++k) b_gr[k] += 2.0 * gr[k] * b_gg;
        }
        // g*_0 = (1 - so) g_0 + so (p3 (w0 - 1) + w0 kin0)
        double b_g[Q];
        double b_p3 = so * (w0 - 1.0) * lg[0], b_kin0 = so * w0 * lg[0];
        double b_rho = 0.0, b_dS = 0.0, b_A[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        double b_F[3] = {0.0, 0.0, 0.0}, b_grho[3] = {0.0, 0.0, 0.0};
        b_g[0] = (1.0 - so) * lg[0];
        // g*_i = (1 - so) g_i + so E_i + fh Fe_i - dS P_i + (so O_i + fh Fo_i), with
        // E = w (p3 + kin0 + 4.5 rho cu^2), O = 3 w rho (c.u) (of opposite sign
        // at opp(i)), Fe = 3 w (c.u)(c.grad rho), Fo = 3 w c.F
        for (int i = 1; i < Q; ++i) {
            const double w = GL::w(i);
            const double cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            const double cu = cx * u[0] + cy * u[1] + cz * u[2];
            const double cr = cx * grho[0] + cy * grho[1] + cz * grho[2];
            double q[5];
            for (int k = 0; k < 5; ++k) q[k] = stress_row<GL, D3>(k, i);
            double P = 0.0;
            for (int k = 0; k < 5; ++k) P += q[k] * A[k];
            const double lb = lg[i];
            b_g[i] = (1.0 - so) * lb;
            const double bE = so * lb, bFe = fh * lb, bO = so * lb, bFo = fh * lb;
            b_p3 += w * bE;
            b_kin0 += w * bE;
            b_rho += 4.5 * w * cu * cu * bE + 3.0 * w * cu * bO;
            const double b_cu = 9.0 * w * rho * cu * bE + 3.0 * w * rho * bO + 3.0 * w * cr * bFe;
            const double b_cr = 3.0 * w * cu * bFe;
            b_u[0] += cx * b_cu;
            b_u[1] += cy * b_cu;
            b_u[2] += cz * b_cu;
            b_grho[0] += cx * b_cr;
            b_grho[1] += cy * b_cr;
            b_grho[2] += cz * b_cr;
            b_F[0] += 3.0 * w * cx * bFo;
            b_F[1] += 3.0 * w * cy * bFo;
            b_F[2] += 3.0 * w * cz * bFo;
            for (int k = 0; k < 5; ++k) b_A[k] += -dS * q[k] * lb;
            b_dS += -P * lb;
        }
        // A (linear in Pi), Pi_kl = m2_kl - rho u_k u_l + (u_k grho_l + u_l grho_k) / 6
        double b_Pi[3][3] = {{0.0}};
        stress_coeffs_T<GL, D3>(b_A, b_Pi);
        double b_m2[3][3] = {{0.0}};
        for (int k = 0; k < 3; ++k)
            for (int l = k; l < 3; ++l) {
                const double b = b_Pi[k][l];
                b_m2[k][l] += b;
                b_rho += -u[k] * u[l] * b;
                b_u[k] += (-rho * u[l] + grho[l] / 6.0) * b;
                b_u[l] += (-rho * u[k] + grho[k] / 6.0) * b;
                b_grho[l] += u[k] / 6.0 * b;
                b_grho[k] += u[l] / 6.0 * b;
            }
        // kin0 = -1.5 rho usq ; p3 = 3 p ; p = cp ((ps - g0) + udr / 2 - 1.5 rho w0 usq)
        double b_usq = -1.5 * rho * b_kin0;
        b_rho += -1.5 * usq * b_kin0;
        const double b_pres = 3.0 * b_p3;
        double b_ps = cp * b_pres;
        b_g[0] += -cp * b_pres;
        const double b_udr = 0.5 * cp * b_pres;
        b_rho += -1.5 * w0 * usq * cp * b_pres;
        b_usq += -1.5 * rho * w0 * cp * b_pres;
        for (int k = 0; k < 3; ++k) {
            b_u[k] += 2.0 * u[k] * b_usq + grho[k] * b_udr;
            b_grho[k] += u[k] * b_udr;
        }
        // u = (j + F / 2) irho ; grho = dR gr ; F = mu gr + rho body + force
        double b_j[3], b_irho = 0.0, b_mu = 0.0;
        for (int k = 0; k < 3; ++k) {
            b_j[k] = irho * b_u[k];
            b_F[k] += 0.5 * irho * b_u[k];
            b_irho += jF[k] * b_u[k];
            b_gr[k] += dR * b_grho[k];
            b_mu += gr[k] * b_F[k];
            b_gr[k] += mu * b_F[k];
            b_rho += ph.body[k] * b_F[k];
        }
        // moments
        moments_T<GL>(b_ps, b_j, b_m2, b_g);
        // mu = beta4 phi (phi - 1)(phi - 1/2) - kappa lap
        const double b_beta4 = b_mu * cub, b_kappa = -b_mu * lap;
        const double b_lap = -ph.kappa * b_mu;
        b_phi += b_mu * ph.beta4 * (3.0 * phi * phi - 3.0 * phi + 0.5);
        // itau = 1 / (3 nu + 1/2), dS = itau - so ; nu ; irho ; rho
        b_phi += phys_T(ph, irho, numu, 3.0 * (-itau * itau * b_dS), b_irho, b_rho);
        // parameters: beta4 = 48 sigma / W, kappa = 1.5 sigma W, anti = 4 / W,
        // itp = 1 / (3 M + 1/2), gfp = 1 - itp / 2
        const double sigma = a.sigma, W = a.W;
        th[0] = b_beta4 * 48.0 / W + b_kappa * 1.5 * W;
        th[1] = -3.0 * itp * itp * (b_itp - 0.5 * b_gfp);
        th[2] = -b_beta4 * 48.0 * sigma / (W * W) + b_kappa * 1.5 * sigma - b_anti * 4.0 / (W * W);

        for (int i = 0; i < Q; ++i) a.og[(size_t)i * nn + n] = b_g[i];
        a.work[n] = b_phi;
        a.work[nn + n] = b_gr[0];
        a.work[2 * nn + n] = b_gr[1];
        a.work[3 * nn + n] = b_gr[2];
        a.work[4 * nn + n] = b_lap;
    }
    block_sums<3, 3>(th, a.partials, wg);
}

// ---------------------------------------------------------------------------
// Liang2014 (Sec. II.D.1): the CH phase field with its own hydrodynamics,
// which read lap(mu_phi) (Eqs. liang2014_velocity_update, liang2_F with F_a),
// a stencil of the field mu_phi = 4 beta phi (phi - 1)(phi - 1/2) - kappa
// lap phi. Passes: phi; mu_phi and lap phi of every node; the reverse sweep,
// which leaves dL/dmu_phi and dL/d(lap mu_phi) of each node; the transpose of
// the mu_phi stencil (a gather, as the phi stencils), which turns them into
// dL/dphi and dL/dlap phi of each node plus the sigma and W terms; then the
// shared stencil transpose and parameter reduction. Workspace values: 0
// dL/dphi, 1-3 dL/dgrad phi, 4 dL/dlap phi, 5 mu_phi, 6 lap phi, 7 dL/dmu_phi,
// 8 dL/dlap mu_phi.

template <class PAIR>
__global__ __launch_bounds__(256) void k_adj_mu_fwd(const AdjArgs a) {
    using GL = typename PAIR::G;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const Nbr nb(a, node_of(n, a));
    const double phi = a.phi[n];
    double lap = 0.0;
    unroll<GL::Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        lap += 6.0 * GL::w(i) * (a.phi[nb.index(GL::c(i, 0), GL::c(i, 1), GL::c(i, 2))] - phi);
    });
    a.work[5 * nn + n] = a.ph.beta4 * phi * (phi - 1.0) * (phi - 0.5) - a.ph.kappa * lap;
    a.work[6 * nn + n] = lap;
}

template <class PAIR>
__global__ __launch_bounds__(256, 2) void k_adj_local_l14(const AdjArgs a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    constexpr int Q = GL::Q, QH = HL::Q;
    constexpr bool D3 = PAIR::dim == 3;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double thM = 0.0;
    if (n < nn) {
        const Node p = node_of(n, a);
        const Phys& ph = a.ph;
        const double* MU = a.work + 5 * nn;
        double g[Q], h[QH], phin[Q], mun[Q];
        for (int i = 0; i < Q; ++i) g[i] = a.fg[(size_t)i * nn + n];
        for (int al = 0; al < QH; ++al) h[al] = a.fh[(size_t)al * nn + n];
        const Nbr nb(a, p);
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            const long long e = nb.index(GL::c(i, 0), GL::c(i, 1), GL::c(i, 2));
            phin[i] = a.phi[e];
            mun[i] = MU[e];
        });
        // ---------------- forward intermediates (as in the step kernel)
        const double phi = phin[0], mu = mun[0];
        double gr[3] = {0.0, 0.0, 0.0}, lapmu = 0.0;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                for (int k = 0; k < 3; ++k) gr[k] += 3.0 * GL::w(i) * GL::c(i, k) * phin[i];
                lapmu += 6.0 * GL::w(i) * (mun[i] - mu);
            }
        });
        const double dR = ph.dRho;
        const double rho = ph.rhoL + phi * dR;
        const double irho = 1.0 / rho;
        const double numu = ph.muL + phi * ph.dMu;
        const double nu = ph.visc_mu ? numu * irho : ph.nuL + phi * ph.dNu;
        const double itau = 1.0 / (3.0 * nu + 0.5);
        double ps, j[3], m2[3][3];
        moments<GL>(g, ps, j, m2);
        const double dM = dR * ph.mob * lapmu;
        const double den = rho - 0.5 * dM;
        const double iden = 1.0 / den;
        double fsb[3], jf[3], u[3], Fp[3], grho[3], Av[3], B[3];
        for (int k = 0; k < 3; ++k) {
            fsb[k] = mu * gr[k] + rho * ph.body[k] + ph.force[k];
            jf[k] = j[k] + 0.5 * fsb[k];
            u[k] = jf[k] * iden;
            Fp[k] = fsb[k] + dM * u[k];
            grho[k] = dR * gr[k];
            Av[k] = grho[k] / 3.0;
            B[k] = Av[k] + Fp[k];
        }
        const double udr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
        const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const double uB = u[0] * B[0] + u[1] * B[1] + u[2] * B[2];
        const double uA = u[0] * Av[0] + u[1] * Av[1] + u[2] * Av[2];
        const double uF = u[0] * Fp[0] + u[1] * Fp[1] + u[2] * Fp[2];
        constexpr double w0 = GL::w(0);
        constexpr double cp = 1.0 / (3.0 * (1.0 - w0));
        const double pres = cp * ((ps - g[0]) + 0.5 * udr - 1.5 * rho * w0 * usq);
        const double so = ph.s_o;
        const double dS = itau - so;
        const double fh = 1.0 - 0.5 * so;
        const double p3 = 3.0 * pres;
        const double kin0 = -1.5 * rho * usq;
        double Pi[3][3];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                Pi[k][l] = m2[k][l] - rho * u[k] * u[l] + 0.5 * (B[k] * u[l] + B[l] * u[k] - 3.0 * uB * u[k] * u[l]);
        double A[5];
        stress_coeffs<GL, D3>(Pi, A);
        const double itp = ph.inv_tau_phi, gfp = ph.g_fac_phi;

        // ---------------- reverse sweep; lambda* gathered through the stream transpose
        double lg[Q], lh[QH];
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            constexpr int cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)GL::opp(i) * nn + n
                                                    : (size_t)i * nn + nb.index(cx, cy, cz);
            lg[i] = a.lg[e];
        });
        unroll<QH>([&](auto J) {
            constexpr int al = J;
            constexpr int cx = HL::c(al, 0), cy = HL::c(al, 1), cz = HL::c(al, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)HL::opp(al) * nn + n
                                                    : (size_t)al * nn + nb.index(cx, cy, cz);
            lh[al] = a.lh[e];
        });
        double b_phi = 0.0, b_u[3] = {0.0, 0.0, 0.0}, b_mu = 0.0;
        double b_itp = 0.0, b_gfp = 0.0;
        // h: the CH collision (Eqs. liang2_geq, liang2_G) with this model's u
        {
            double pu[3], pup[3], b_pu[3], b_pup[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < 3; ++k) {
                pu[k] = phi * u[k];
                pup[k] = a.fpu[(size_t)k * nn + n];
                b_pu[k] = a.lpu[(size_t)k * nn + n];
            }
            unroll<QH>([&](auto J) {
                constexpr int al = J;
                constexpr double w = HL::w(al);
                constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
                const double lb = lh[al];
                const double bheq = itp * lb;
                double heq, G = 0.0;
                if constexpr (al == 0) {
                    heq = phi + (w - 1.0) * ph.eta * mu;
                    b_phi += bheq;
                    b_mu += (w - 1.0) * ph.eta * bheq;
                } else {
                    const double ep = ex * pu[0] + ey * pu[1] + ez * pu[2];
                    const double eq = ex * pup[0] + ey * pup[1] + ez * pup[2];
                    heq = w * ph.eta * mu + 3.0 * w * ep;
                    G = 3.0 * w * (ep - eq);
                    b_mu += w * ph.eta * bheq;
                    const double t = 3.0 * w * (bheq + gfp * lb);
                    const double tp = 3.0 * w * gfp * lb;
                    b_pu[0] += ex * t;
                    b_pu[1] += ey * t;
                    b_pu[2] += ez * t;
                    b_pup[0] -= ex * tp;
                    b_pup[1] -= ey * tp;
                    b_pup[2] -= ez * tp;
                }
                b_itp += (heq - h[al]) * lb;
                b_gfp += G * lb;
            });
            for (int k = 0; k < 3; ++k) {
                b_phi += u[k] * b_pu[k];
                b_u[k] += phi * b_pu[k];
                a.opu[(size_t)k * nn + n] = b_pup[k];
            }
        }
        // f*_i = (1 - so) f_i + so feq_i + fh F_i - dS P_i with
        // feq_i = w (p3 + kin0 + 4.5 rho cu^2 + 3 rho cu) - [i = 0] p3,
        // F_i = 3 ((c.A - u.A) Gam_i + (c.F' - u.F')(w + Gam_i)),
        // Gam_i = w (3 cu + 4.5 cu^2 - 1.5 u.u)
        double b_g[Q];
        double b_p3 = 0.0, b_kin0 = 0.0, b_rho = 0.0, b_dS = 0.0, b_usq = 0.0;
        double b_uA = 0.0, b_uF = 0.0, b_A[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        double b_Fp[3] = {0.0, 0.0, 0.0}, b_Av[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double w = GL::w(i);
            const double cx = GL::c(i, 0), cy = GL::c(i, 1), cz = GL::c(i, 2);
            const double cu = cx * u[0] + cy * u[1] + cz * u[2];
            const double cF = cx * Fp[0] + cy * Fp[1] + cz * Fp[2];
            const double cA = cx * Av[0] + cy * Av[1] + cz * Av[2];
            const double Gam = w * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            double q[5];
            for (int k = 0; k < 5; ++k) q[k] = stress_row<GL, D3>(k, i);
            double P = 0.0;
            for (int k = 0; k < 5; ++k) P += q[k] * A[k];
            const double lb = lg[i];
            b_g[i] = (1.0 - so) * lb;
            const double bfeq = so * lb, bF = fh * lb;
            b_p3 += (i == 0 ? w - 1.0 : w) * bfeq;
            b_kin0 += w * bfeq;
            b_rho += w * (4.5 * cu * cu + 3.0 * cu) * bfeq;
            double b_cu = w * rho * (9.0 * cu + 3.0) * bfeq;
            const double b_cA = 3.0 * Gam * bF, b_cF = 3.0 * (w + Gam) * bF;
            b_uA += -3.0 * Gam * bF;
            b_uF += -3.0 * (w + Gam) * bF;
            const double b_Gam = 3.0 * ((cA - uA) + (cF - uF)) * bF;
            b_cu += w * (3.0 + 9.0 * cu) * b_Gam;
            b_usq += -1.5 * w * b_Gam;
            b_u[0] += cx * b_cu;
            b_u[1] += cy * b_cu;
            b_u[2] += cz * b_cu;
            b_Fp[0] += cx * b_cF;
            b_Fp[1] += cy * b_cF;
            b_Fp[2] += cz * b_cF;
            b_Av[0] += cx * b_cA;
            b_Av[1] += cy * b_cA;
            b_Av[2] += cz * b_cA;
            for (int k = 0; k < 5; ++k) b_A[k] += -dS * q[k] * lb;
            b_dS += -P * lb;
        }
        // A (linear in Pi); Pi_kl = m2_kl - rho u_k u_l + (B_k u_l + B_l u_k - 3 (u.B) u_k u_l) / 2
        double b_Pi[3][3] = {{0.0}};
        stress_coeffs_T<GL, D3>(b_A, b_Pi);
        double b_m2[3][3] = {{0.0}}, b_B[3] = {0.0, 0.0, 0.0}, b_uB = 0.0;
        for (int k = 0; k < 3; ++k)
            for (int l = k; l < 3; ++l) {
                const double b = b_Pi[k][l];
                b_m2[k][l] += b;
                b_rho += -u[k] * u[l] * b;
                b_u[k] += (-rho * u[l] + 0.5 * B[l] - 1.5 * uB * u[l]) * b;
                b_u[l] += (-rho * u[k] + 0.5 * B[k] - 1.5 * uB * u[k]) * b;
                b_B[k] += 0.5 * u[l] * b;
                b_B[l] += 0.5 * u[k] * b;
                b_uB += -1.5 * u[k] * u[l] * b;
            }
        // kin0, p3 = 3 p, p = cp ((ps - g0) + udr / 2 - 1.5 rho w0 usq)
        b_rho += -1.5 * usq * b_kin0;
        b_usq += -1.5 * rho * b_kin0;
        const double b_pres = 3.0 * b_p3;
        const double b_ps = cp * b_pres;
        b_g[0] += -cp * b_pres;
        const double b_udr = 0.5 * cp * b_pres;
        b_rho += -1.5 * w0 * usq * cp * b_pres;
        b_usq += -1.5 * rho * w0 * cp * b_pres;
        // uB, uA, uF, B = A + F', usq, udr
        double b_grho[3], b_fsb[3], b_dM = 0.0;
        for (int k = 0; k < 3; ++k) {
            b_u[k] += B[k] * b_uB + Av[k] * b_uA + Fp[k] * b_uF + 2.0 * u[k] * b_usq + grho[k] * b_udr;
            b_B[k] += u[k] * b_uB;
            b_Av[k] += u[k] * b_uA + b_B[k];
            b_Fp[k] += u[k] * b_uF + b_B[k];
            b_grho[k] = u[k] * b_udr + b_Av[k] / 3.0;
            // F' = fsb + dM u
            b_fsb[k] = b_Fp[k];
            b_dM += u[k] * b_Fp[k];
            b_u[k] += dM * b_Fp[k];
        }
        // u = (j + fsb / 2) / den, den = rho - dM / 2
        double b_j[3], b_iden = 0.0;
        for (int k = 0; k < 3; ++k) {
            b_j[k] = iden * b_u[k];
            b_fsb[k] += 0.5 * iden * b_u[k];
            b_iden += jf[k] * b_u[k];
        }
        const double b_den = -iden * iden * b_iden;
        b_rho += b_den;
        b_dM += -0.5 * b_den;
        // dM = dR M lap(mu) ; fsb = mu gr + rho body + force ; grho = dR gr
        const double b_lapmu = dR * ph.mob * b_dM;
        thM = dR * lapmu * b_dM;
        double b_gr[3];
        for (int k = 0; k < 3; ++k) {
            b_mu += gr[k] * b_fsb[k];
            b_gr[k] = mu * b_fsb[k] + dR * b_grho[k];
            b_rho += ph.body[k] * b_fsb[k];
        }
        // moments
        moments_T<GL>(b_ps, b_j, b_m2, b_g);
        // itau, nu, irho, rho
        b_phi += phys_T(ph, irho, numu, 3.0 * (-itau * itau * b_dS), 0.0, b_rho);
        // tau_phi = 3 M / eta + 1/2 (itp, gfp = 1 - itp / 2); M also in F_a
        thM += -3.0 / ph.eta * itp * itp * (b_itp - 0.5 * b_gfp);

        for (int i = 0; i < Q; ++i) a.og[(size_t)i * nn + n] = b_g[i];
        a.work[n] = b_phi;
        a.work[nn + n] = b_gr[0];
        a.work[2 * nn + n] = b_gr[1];
        a.work[3 * nn + n] = b_gr[2];
        a.work[7 * nn + n] = b_mu;
        a.work[8 * nn + n] = b_lapmu;
    }
    const double th[3] = {0.0, thM, 0.0};
    block_sums<3, 3>(th, a.partials, wg);
}

// transpose of the mu_phi stencil: dL/dmu_phi(y) = work[7](y) plus lap^T of
// work[8]; then mu_phi = beta4 phi (phi - 1)(phi - 1/2) - kappa lap phi gives
// dL/dphi(y) += beta4 (3 phi^2 - 3 phi + 1/2) dL/dmu_phi, dL/dlap phi(y) =
// -kappa dL/dmu_phi, and the sigma and W terms (beta4 = 48 sigma / W, kappa =
// 1.5 sigma W), added to the sweep's block partials
template <class PAIR>
__global__ __launch_bounds__(256) void k_adj_mu_l14(const AdjArgs a) {
    using GL = typename PAIR::G;
    constexpr int Q = GL::Q;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double th[3] = {0.0, 0.0, 0.0};
    if (n < nn) {
        const double* blap = a.work + 8 * nn;
        double acc = a.work[7 * nn + n] - 6.0 * (1.0 - GL::w(0)) * blap[n];
        const Nbr nb(a, node_of(n, a));
        unroll<Q - 1>([&](auto I) {
            constexpr int i = I + 1;
            constexpr int c0 = GL::c(i, 0), c1 = GL::c(i, 1), c2 = GL::c(i, 2);
            constexpr double w6 = 6.0 * GL::w(i);
            if (!nb.beyond(-c0, -c1, -c2)) acc += w6 * blap[nb.index(-c0, -c1, -c2)];
            unroll<3>([&](auto K) {
                constexpr int k = K;
                constexpr int ck = k == 0 ? c0 : (k == 1 ? c1 : c2);
                if constexpr (ck != 0) {
                    if (nb.bnd[k][ck + 1]) {
                        constexpr int dx = k == 0 ? 0 : -c0, dy = k == 1 ? 0 : -c1, dz = k == 2 ? 0 : -c2;
                        if (!nb.beyond(dx, dy, dz)) acc += w6 * blap[nb.index(dx, dy, dz)];
                    }
                }
            });
        });
        const Phys& ph = a.ph;
        const double phi = a.phi[n], lap = a.work[6 * nn + n];
        const double cub = phi * (phi - 1.0) * (phi - 0.5);
        a.work[n] += ph.beta4 * (3.0 * phi * phi - 3.0 * phi + 0.5) * acc;
        a.work[4 * nn + n] = -ph.kappa * acc;
        const double sigma = a.sigma, W = a.W;
        th[0] = acc * (cub * 48.0 / W - lap * 1.5 * W);
        th[2] = -acc * (cub * 48.0 * sigma / (W * W) + lap * 1.5 * sigma);
    }
    block_sums<3, 3, true>(th, a.partials, wg);
}

// pass 3: transpose of grad phi(x) = 3 sum w c phi(src(x, i)) and
// lap phi(x) = 6 sum w (phi(src(x, i)) - phi(x)), src = periodic image or wall
// mirror of x + c_i, as a gather at y over {x : src(x, i) = y}; every h
// population of y receives that plus dL/dphi(y), and its direct term
// (1 - 1/tau_phi) lambda*_h (the h stream transpose of lambda_h^{n+1},
// gathered here rather than written by the sweep and read back).
// MODE 0: that, into lambda_h^n (AC, CH). MODE 1: the transpose of the
// Laplacian alone, for the adjoint of the CH initialisation (mu_phi(phi0) in
// h_eq): dL/dphi0 = work[0] + lap^T(work[4]). MODE 2 (nonlocal model): the
// total dL/dphi* into work[0] (in place: only this node reads it), the
// nonlocal correction's transpose and the h populations follow.
// The sum of the sweep's per-workgroup parameter partials [nb][3], added into
// out, by one 256-thread workgroup in a fixed order (bit-reproducible):
// strided per-thread sums, a shuffle tree within each wave, the four waves in
// order.
__device__ __forceinline__ void params_fold(const double* part, int nb, double* out) {
    __shared__ double wsum[3][4];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 3; ++k) s[k] += part[(size_t)b * 3 + k];
    for (int k = 0; k < 3; ++k)
        for (int off = 32; off >= 1; off >>= 1) s[k] += __shfl_down(s[k], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) wsum[k][threadIdx.x >> 6] = s[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] += ((wsum[k][0] + wsum[k][1]) + wsum[k][2]) + wsum[k][3];
}

constexpr int ST_STEP = 0, ST_INIT = 1, ST_NL = 2;
template <class PAIR, int MODE, class R = double>
__global__ __launch_bounds__(256) void k_adj_stencil(const AdjArgsT<R> a) {
    constexpr bool INIT = MODE == ST_INIT;
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    constexpr int Q = GL::Q;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    // the sweep (the previous launch) has written every partial: the first
    // workgroup to start sums them while the others run (in place of a launch
    // of its own); every thread of the workgroup takes part, so this comes
    // before the early return
    if constexpr (MODE == ST_STEP)
        if (a.dparams && blockIdx.x == 0) params_fold(a.partials, (int)gridDim.x, a.dparams);
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const Node p = node_of(n, a);
    const R* bphi = a.work;
    const R* bgr = a.work + nn;
    const R* blap = a.work + 4 * nn;
    R acc = bphi[n] - R(6.0) * (R(1.0) - R(GL::w(0))) * blap[n];
    const Nbr nb(a, p);
    // lambda_h^{n+1} through the transposed h streaming, gathered before any
    // store (a store may alias it, so later loads could not pass it)
    R lhv[HL::Q];
    if constexpr (MODE == ST_STEP) {
        unroll<HL::Q>([&](auto J) {
            constexpr int al = J;
            constexpr int cx = HL::c(al, 0), cy = HL::c(al, 1), cz = HL::c(al, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)HL::opp(al) * nn + n
                                                    : (size_t)al * nn + nb.index(cx, cy, cz);
            lhv[al] = a.lh[e];
        });
    }
    unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        constexpr int c0 = GL::c(i, 0), c1 = GL::c(i, 1), c2 = GL::c(i, 2);
        constexpr R w3 = R(3.0) * R(GL::w(i)), w6 = R(6.0) * R(GL::w(i));
        // the terms of x's stencil that reach y (zero components skipped)
        auto contrib = [&](long long x) {
            R t = w6 * blap[x];
            if constexpr (!INIT && c0 != 0) t += (w3 * c0) * bgr[x];
            if constexpr (!INIT && c1 != 0) t += (w3 * c1) * bgr[nn + x];
            if constexpr (!INIT && c2 != 0) t += (w3 * c2) * bgr[2 * nn + x];
            acc += t;
        };
        // x = y - c_i (no wall crossed)
        if (!nb.beyond(-c0, -c1, -c2)) contrib(nb.index(-c0, -c1, -c2));
        // at a wall layer (y + c_i beyond the wall along axis k): x on the same
        // layer whose x + c_i is mirrored onto y
        unroll<3>([&](auto K) {
            constexpr int k = K;
            constexpr int ck = k == 0 ? c0 : (k == 1 ? c1 : c2);
            if constexpr (ck != 0) {
                if (nb.bnd[k][ck + 1]) {
                    constexpr int dx = k == 0 ? 0 : -c0, dy = k == 1 ? 0 : -c1, dz = k == 2 ? 0 : -c2;
                    if (!nb.beyond(dx, dy, dz)) contrib(nb.index(dx, dy, dz));
                }
            }
        });
    });
    if constexpr (INIT) {
        a.dphi0[n] = acc;
        return;
    }
    if constexpr (MODE == ST_NL) {
        a.work[n] = acc;
        return;
    }
    const R itp1 = R(1.0) - R(a.ph.inv_tau_phi);
    unroll<HL::Q>([&](auto J) {
        constexpr int al = J;
        a.oh[(size_t)al * nn + n] = itp1 * lhv[al] + acc;
    });
}

// one workgroup, fixed summation order (bit-reproducible); 1024 threads so the
// per-thread strided sums are short
constexpr int PARAMS_THREADS = 1024;
__global__ __launch_bounds__(PARAMS_THREADS) void k_adj_params(const double* part, int nb, double* out) {
    __shared__ double red[3][PARAMS_THREADS];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += PARAMS_THREADS)
        for (int k = 0; k < 3; ++k) s[k] += part[(size_t)b * 3 + k];
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int st = PARAMS_THREADS / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] += red[k][0];
}

// ---------------------------------------------------------------------------
// nonlocal model (Eqs. nonlocalAC, lagrange_multiplier, chai_G, Hu_G): the
// step uses phi* = phi + (1 - lam) R(phi, gamma) / 2 in place of phi = sum h,
// R = M (gamma phi (1 - phi) - (32 / W^2) phi (phi - 1)(phi - 1/2)), gamma =
// sum (32 / W^2) phi (phi - 1)(phi - 1/2) / sum phi (1 - phi) over all nodes
// (0 when that denominator vanishes). Its transpose needs two global sums:
// gamma of the state, and dL/dgamma = sum_x dL/dR(x) M phi(x) (1 - phi(x)).

// phi = sum h into work[6], partial sums of gamma's numerator and denominator
__global__ __launch_bounds__(256) void k_adj_phi_nl(const AdjArgs a) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};   // the third slot is unused (zero)
    if (n < nn) {
        double s = a.fh[n];
        for (int al = 1; al < a.qh; ++al) s += a.fh[(size_t)al * nn + n];
        a.work[6 * nn + n] = s;
        v[0] = a.ph.w32 * (s - 1.0) * s * (s - 0.5);
        v[1] = s * (1.0 - s);
    }
    block_sums<3, 4>(v, a.nlpart, wg);
}

// one workgroup, fixed order. MODE 0: gamma = num / den (0 if den = 0) and
// den into nls[0], nls[1]. MODE 1: dL/dgamma into nls[2]; the source's M and
// W terms added into dparams[1], dparams[2] (if given)
__global__ __launch_bounds__(1024) void k_adj_nlred(const double* part, int nb, int mode, double* nls,
                                                    double* dparams) {
    __shared__ double red[3][1024];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 1024)
        for (int k = 0; k < 3; ++k) s[k] += part[(size_t)b * 4 + k];
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int st = 512; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == 0) {
            nls[0] = red[1][0] != 0.0 ? red[0][0] / red[1][0] : 0.0;
            nls[1] = red[1][0];
        } else {
            nls[2] = red[0][0];
            if (dparams) {
                dparams[1] += red[1][0];
                dparams[2] += red[2][0];
            }
        }
    }
}

__device__ __forceinline__ double nl_R(const Phys& ph, double p, double gam) {
    return ph.mob * (gam * p * (1.0 - p) - ph.w32 * (p - 1.0) * p * (p - 0.5));
}

// phi* of every node into the workspace's phi
__global__ __launch_bounds__(256) void k_adj_phistar(const AdjArgs a) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double p = a.work[6 * nn + n];
    a.phi[n] = p + 0.5 * (1.0 - a.ph.lam) * nl_R(a.ph, p, a.nls[0]);
}

// transpose of phi* = phi + (1 - lam) R / 2 at each node, without gamma's
// global term: from dL/dphi* (work[0], or the seed dphi) and the collision's
// direct dL/dR (work[5], or none for the seed), dL/dR = direct + (1 - lam)
// dL/dphi* / 2 and dL/dphi = dL/dphi* + dL/dR dR/dphi into work[0]; block
// partials of dL/dgamma, dL/dM = sum dL/dR R / M and dL/dW = sum dL/dR
// (-2 R / W) (R scales with 32 / W^2, gamma included)
__global__ __launch_bounds__(256) void k_adj_nl_map(const AdjArgs a, const double* dphis, const double* bRd) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (n < nn) {
        const Phys& ph = a.ph;
        const double p = a.work[6 * nn + n], gam = a.nls[0];
        const double acc = dphis[n];
        const double bR = (bRd ? bRd[n] : 0.0) + 0.5 * (1.0 - ph.lam) * acc;
        const double well = p * (1.0 - p);
        const double Rm = gam * well - ph.w32 * (p - 1.0) * p * (p - 0.5);   // R / M
        const double dR = ph.mob * (gam * (1.0 - 2.0 * p) - ph.w32 * (3.0 * p * p - 3.0 * p + 0.5));
        a.work[n] = acc + bR * dR;
        v[0] = bR * ph.mob * well;
        v[1] = bR * Rm;
        v[2] = bR * (-2.0 * ph.mob * Rm / a.W);
    }
    block_sums<3, 4>(v, a.nlpart, wg);
}

// dL/dphi = work[0] + dL/dgamma dgamma/dphi, dgamma/dphi = ((32 / W^2)
// (3 phi^2 - 3 phi + 1/2) - gamma (1 - 2 phi)) / den, into every h population:
// SEED: lam_h = that (lam_g = 0); otherwise oh = that plus the direct term
// (1 - 1/tau_phi) lambda*_h (the h stream transpose of lambda_h^{n+1})
template <class PAIR, bool SEED>
__global__ __launch_bounds__(256) void k_adj_nl_final(const AdjArgs a, double* lam_g, double* lam_h) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const Phys& ph = a.ph;
    const double p = a.work[6 * nn + n], gam = a.nls[0], den = a.nls[1];
    const double dgam = den != 0.0 ? (ph.w32 * (3.0 * p * p - 3.0 * p + 0.5) - gam * (1.0 - 2.0 * p)) / den : 0.0;
    const double t = a.work[n] + a.nls[2] * dgam;
    if constexpr (SEED) {
        for (int i = 0; i < GL::Q; ++i) lam_g[(size_t)i * nn + n] = 0.0;
        for (int al = 0; al < HL::Q; ++al) lam_h[(size_t)al * nn + n] = t;
    } else {
        const Nbr nb(a, node_of(n, a));
        const double itp1 = 1.0 - ph.inv_tau_phi;
        double lhv[HL::Q];   // gathered before any store (see the stencil pass)
        unroll<HL::Q>([&](auto J) {
            constexpr int al = J;
            constexpr int cx = HL::c(al, 0), cy = HL::c(al, 1), cz = HL::c(al, 2);
            const size_t e = nb.beyond(cx, cy, cz) ? (size_t)HL::opp(al) * nn + n
                                                    : (size_t)al * nn + nb.index(cx, cy, cz);
            lhv[al] = a.lh[e];
        });
        unroll<HL::Q>([&](auto J) {
            constexpr int al = J;
            a.oh[(size_t)al * nn + n] = itp1 * lhv[al] + t;
        });
    }
}

// dL/dphi0 through the equilibrium initialisation h = h_eq(phi0, u0),
// g = g_eq(3 p0 / rho(phi0), u0); MODEL 0 AC, 2 nonlocal, 3 Liang2018
template <class PAIR, int MODEL, class R = double>
__global__ __launch_bounds__(256) void k_adj_init(const AdjInitArgsT<R> a) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    R u[3] = {R(0.0), R(0.0), R(0.0)};
    if (a.u0) {
        u[0] = a.u0[n];
        u[1] = a.u0[nn + n];
        if (PAIR::dim == 3) u[2] = a.u0[2 * nn + n];
    }
    const R usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    R s = R(0.0);
    for (int al = 0; al < HL::Q; ++al) {
        const R eu = HL::c(al, 0) * u[0] + HL::c(al, 1) * u[1] + HL::c(al, 2) * u[2];
        // Eq. fakhari_geq (AC) or Eqs. Chai_geq, liang_geq (first order in u)
        const R dh = MODEL == 2 || MODEL == 3 ? R(1.0) + R(3.0) * eu : R(1.0) + R(3.0) * eu + R(4.5) * eu * eu - R(1.5) * usq;
        s += a.lh[(size_t)al * nn + n] * R(HL::w(al)) * dh;
    }
    if constexpr (MODEL == 3) {
        // Eq. liang_feq: (p0/c_s^2)(w - [i = 0]) + rho(phi0) w (3 c.u + 4.5 (c.u)^2
        // - 1.5 u.u); (phi u) = phi0 u0
        R sg = R(0.0);
        for (int i = 0; i < GL::Q; ++i) {
            const R cu = GL::c(i, 0) * u[0] + GL::c(i, 1) * u[1] + GL::c(i, 2) * u[2];
            sg += a.lg[(size_t)i * nn + n] * R(GL::w(i)) * (R(3.0) * cu + R(4.5) * cu * cu - R(1.5) * usq);
        }
        s += R(a.ph.dRho) * sg;
        for (int k = 0; k < 3; ++k) s += a.lpu[(size_t)k * nn + n] * u[k];
    } else if (a.p0) {
        const R phi = R(a.phi0[n]);
        const R rho = R(a.ph.rhoL) + phi * R(a.ph.dRho);
        const R dps = -R(3.0) * R(a.p0[n]) * R(a.ph.dRho) / (rho * rho);
        for (int i = 0; i < GL::Q; ++i) s += a.lg[(size_t)i * nn + n] * R(GL::w(i)) * dps;
    }
    a.dphi0[n] = s;
}

// adjoint of the CH initialisation h = h_eq(phi0, mu_phi(phi0), u0) (Eq.
// liang2_geq with mu_phi of Eq. chemical_potential), g = g_eq(3 p0 / rho(phi0),
// u0) (MODEL 1; Liang2014, MODEL 4: f = f_eq of Eq. liang2_feq at rho(phi0)),
// (phi u) = phi0 u0: the local part of dL/dphi0 into work[0],
// dL/d(lap phi0) into work[4] (the stencil pass in init mode adds its
// transpose), and the sigma and W terms of mu_phi into the block partials
template <class PAIR, int MODEL, class R = double>
__global__ __launch_bounds__(256) void k_adj_init_ch(const AdjArgsT<R> a, const double* phi0, const double* u0,
                                                     const double* p0) {
    using GL = typename PAIR::G;
    using HL = typename PAIR::H;
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const int wg = xcd_block();
    const long long n = (long long)wg * blockDim.x + threadIdx.x;
    double th[3] = {0.0, 0.0, 0.0};
    if (n < nn) {
        const Phys& ph = a.ph;
        const Nbr nb(a, node_of(n, a));
        const double phi = phi0[n];
        double lap = 0.0;
        unroll<GL::Q - 1>([&](auto I) {
            constexpr int i = I + 1;
            lap += 6.0 * GL::w(i) * (phi0[nb.index(GL::c(i, 0), GL::c(i, 1), GL::c(i, 2))] - phi);
        });
        double u[3] = {0.0, 0.0, 0.0};
        if (u0) {
            u[0] = u0[n];
            u[1] = u0[nn + n];
            if (PAIR::dim == 3) u[2] = u0[2 * nn + n];
        }
        const double cub = phi * (phi - 1.0) * (phi - 0.5);
        // heq_0 = phi + (w_0 - 1) eta mu, heq_a = w_a eta mu + 3 w_a e_a . (phi u)
        double s = a.lh[n], cmu = -(double)a.lh[n];
        unroll<HL::Q>([&](auto J) {
            constexpr int al = J;
            const double lb = a.lh[(size_t)al * nn + n];
            cmu += HL::w(al) * lb;
            if constexpr (al > 0) {
                constexpr int ex = HL::c(al, 0), ey = HL::c(al, 1), ez = HL::c(al, 2);
                s += 3.0 * HL::w(al) * (ex * u[0] + ey * u[1] + ez * u[2]) * lb;
            }
        });
        cmu *= ph.eta;   // dL/dmu_phi
        for (int k = 0; k < 3; ++k) s += a.lpu[(size_t)k * nn + n] * u[k];
        s += cmu * ph.beta4 * (3.0 * phi * phi - 3.0 * phi + 0.5);
        if constexpr (MODEL == 4) {
            // Eq. liang2_feq: the kinetic part rho(phi0) w (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
            const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            double sg = 0.0;
            for (int i = 0; i < GL::Q; ++i) {
                const double cu = GL::c(i, 0) * u[0] + GL::c(i, 1) * u[1] + GL::c(i, 2) * u[2];
                sg += a.lg[(size_t)i * nn + n] * GL::w(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            }
            s += ph.dRho * sg;
        } else if (p0) {
            const double rho = ph.rhoL + phi * ph.dRho;
            const double dps = -3.0 * p0[n] * ph.dRho / (rho * rho);
            for (int i = 0; i < GL::Q; ++i) s += a.lg[(size_t)i * nn + n] * GL::w(i) * dps;
        }
        a.work[n] = R(s);
        a.work[4 * nn + n] = R(-ph.kappa * cmu);
        // beta4 = 48 sigma / W, kappa = 1.5 sigma W
        const double sigma = a.sigma, W = a.W;
        th[0] = cmu * (cub * 48.0 / W - lap * 1.5 * W);
        th[2] = -cmu * (cub * 48.0 * sigma / (W * W) + lap * 1.5 * sigma);
    }
    block_sums<3, 3>(th, a.partials, wg);
}

// seed of the adjoint from dL/dphi of a state: phi = sum_a h_a (Eq.
// fakhari_phi_update) gives dL/dh_a = dL/dphi for every a, and dL/dg = 0
template <class R>
__global__ __launch_bounds__(256) void k_adj_seed(const R* dphi, R* lg, R* lh, long long nn, int qg, int qh) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const R v = dphi[n];
    for (int i = 0; i < qg; ++i) lg[(size_t)i * nn + n] = R(0);
    for (int a = 0; a < qh; ++a) lh[(size_t)a * nn + n] = v;
}

hipError_t launch_adjoint_seed(const double* dphi, double* lg, double* lh, long long nn, int qg, int qh,
                               hipStream_t st) {
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_adj_seed<double>, grid, block, 0, st, dphi, lg, lh, nn, qg, qh);
    return hipGetLastError();
}

hipError_t launch_adjoint(int lattice, int model, const AdjArgs& a, double* dparams, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    if (model == 2) {
        // phi = sum h, gamma, phi*
        hipLaunchKernelGGL(k_adj_phi_nl, grid, block, 0, st, a);
        hipLaunchKernelGGL(k_adj_nlred, dim3(1), dim3(1024), 0, st, (const double*)a.nlpart, (int)grid.x, 0, a.nls,
                           (double*)nullptr);
        hipLaunchKernelGGL(k_adj_phistar, grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL(k_adj_phi<double>, grid, block, 0, st, a);
    }
    auto go = [&](auto pair) {
        using P_ = decltype(pair);
        if (model == 2) {
            hipLaunchKernelGGL((k_adj_local<P_, 2>), grid, block, 0, st, a);
            hipLaunchKernelGGL((k_adj_stencil<P_, ST_NL>), grid, block, 0, st, a);
            hipLaunchKernelGGL(k_adj_nl_map, grid, block, 0, st, a, (const double*)a.work,
                               (const double*)(a.work + 5 * nn));
            hipLaunchKernelGGL(k_adj_nlred, dim3(1), dim3(1024), 0, st, (const double*)a.nlpart, (int)grid.x, 1,
                               a.nls, dparams);
            hipLaunchKernelGGL((k_adj_nl_final<P_, false>), grid, block, 0, st, a, (double*)nullptr,
                               (double*)nullptr);
            return;
        }
        if (model == 1) {
            hipLaunchKernelGGL((k_adj_local<P_, 1>), grid, block, 0, st, a);
        } else if (model == 3) {
            hipLaunchKernelGGL((k_adj_local_l18<P_>), grid, block, 0, st, a);
        } else if (model == 4) {
            hipLaunchKernelGGL((k_adj_mu_fwd<P_>), grid, block, 0, st, a);
            hipLaunchKernelGGL((k_adj_local_l14<P_>), grid, block, 0, st, a);
            hipLaunchKernelGGL((k_adj_mu_l14<P_>), grid, block, 0, st, a);
        } else {
            hipLaunchKernelGGL((k_adj_local<P_, 0>), grid, block, 0, st, a);
        }
        // the stencil pass also sums the sweep's parameter partials
        AdjArgs b = a;
        b.dparams = dparams;
        hipLaunchKernelGGL((k_adj_stencil<P_, ST_STEP>), grid, block, 0, st, b);
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    if (model == 2 && dparams)
        hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(PARAMS_THREADS), 0, st, a.partials, (int)grid.x, dparams);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(int lattice, int model, const AdjInitArgs& a, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    auto go = [&](auto pair) {
        using P_ = decltype(pair);
        if (model == 2) hipLaunchKernelGGL((k_adj_init<P_, 2>), grid, block, 0, st, a);
        else if (model == 3) hipLaunchKernelGGL((k_adj_init<P_, 3>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_adj_init<P_, 0>), grid, block, 0, st, a);
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    return hipGetLastError();
}

hipError_t launch_adjoint_seed_nl(int lattice, const AdjArgs& a, const double* dphi, double* lam_g, double* lam_h,
                                  double* dparams, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_adj_phi_nl, grid, block, 0, st, a);
    hipLaunchKernelGGL(k_adj_nlred, dim3(1), dim3(1024), 0, st, (const double*)a.nlpart, (int)grid.x, 0, a.nls,
                       (double*)nullptr);
    hipLaunchKernelGGL(k_adj_nl_map, grid, block, 0, st, a, dphi, (const double*)nullptr);
    hipLaunchKernelGGL(k_adj_nlred, dim3(1), dim3(1024), 0, st, (const double*)a.nlpart, (int)grid.x, 1, a.nls,
                       dparams);
    auto go = [&](auto pair) {
        using P_ = decltype(pair);
        hipLaunchKernelGGL((k_adj_nl_final<P_, true>), grid, block, 0, st, a, lam_g, lam_h);
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    return hipGetLastError();
}

hipError_t launch_adjoint_init_ch(int lattice, int model, const AdjArgs& a, const double* phi0, const double* u0,
                                  const double* p0, double* dparams, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    auto go = [&](auto pair) {
        using P_ = decltype(pair);
        if (model == 4) hipLaunchKernelGGL((k_adj_init_ch<P_, 4>), grid, block, 0, st, a, phi0, u0, p0);
        else hipLaunchKernelGGL((k_adj_init_ch<P_, 1>), grid, block, 0, st, a, phi0, u0, p0);
        hipLaunchKernelGGL((k_adj_stencil<P_, ST_INIT>), grid, block, 0, st, a);
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    if (dparams) hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(PARAMS_THREADS), 0, st, a.partials, (int)grid.x, dparams);
    return hipGetLastError();
}

// float32 adjoint of the AC step: the same passes in float32 arithmetic on
// float32 arrays; the parameter partials and their reduction stay float64
hipError_t launch_adjoint_f32(int lattice, int model, const AdjArgsT<float>& a, double* dparams, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_adj_phi<float>, grid, block, 0, st, a);
    auto go = [&](auto pair) {
        using P_ = decltype(pair);
        if (model == 1) hipLaunchKernelGGL((k_adj_local<P_, 1, float>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_adj_local<P_, 0, float>), grid, block, 0, st, a);
        AdjArgsT<float> b = a;
        b.dparams = dparams;
        hipLaunchKernelGGL((k_adj_stencil<P_, ST_STEP, float>), grid, block, 0, st, b);
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    return hipGetLastError();
}

hipError_t launch_adjoint_seed_f32(const float* dphi, float* lg, float* lh, long long nn, int qg, int qh,
                                   hipStream_t st) {
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_adj_seed<float>, grid, block, 0, st, dphi, lg, lh, nn, qg, qh);
    return hipGetLastError();
}

hipError_t launch_adjoint_init_ch_f32(int lattice, const AdjArgsT<float>& a, const double* phi0, const double* u0,
                                      const double* p0, double* dparams, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    auto go = [&](auto pair) {
        using P_ = decltype(pair);
        hipLaunchKernelGGL((k_adj_init_ch<P_, 1, float>), grid, block, 0, st, a, phi0, u0, p0);
        hipLaunchKernelGGL((k_adj_stencil<P_, ST_INIT, float>), grid, block, 0, st, a);
    };
    if (lattice == 0) go(Pair2D{});
    else if (lattice == 1) go(Pair3D{});
    else go(Pair3D27{});
    if (dparams) hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(PARAMS_THREADS), 0, st, a.partials, (int)grid.x, dparams);
    return hipGetLastError();
}

hipError_t launch_adjoint_init_f32(int lattice, const AdjInitArgsT<float>& a, hipStream_t st) {
    const long long nn = (long long)a.nx * a.ny * a.nz;
    const dim3 grid((unsigned)((nn + 255) / 256)), block(256);
    if (lattice == 0) hipLaunchKernelGGL((k_adj_init<Pair2D, 0, float>), grid, block, 0, st, a);
    else if (lattice == 1) hipLaunchKernelGGL((k_adj_init<Pair3D, 0, float>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_adj_init<Pair3D27, 0, float>), grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace pfk
