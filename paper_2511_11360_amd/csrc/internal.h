// Internal interface between the C ABI (pflbm.cpp) and the kernels
// (kernels.hip). Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pfk {

constexpr int BLOCK = 256;      // threads per workgroup (step tiles 0-2, reductions)
// step tiles (x nodes, y rows, threads) by tile index; fields / diagnostics
// use tile 0; tile 3 is a 1024-thread workgroup
constexpr int NTILES = 5;
constexpr int TILE_NX[NTILES] = {64, 128, 256, 256, 128};
constexpr int TILE_NY[NTILES] = {4, 2, 1, 4, 8};
constexpr int TILE_THREADS[NTILES] = {256, 256, 256, 1024, 1024};
constexpr int NDIAG = 12;       // per-block partial diagnostics (see kernels.hip)
constexpr int GAMMA_ZB = 16;    // z planes per workgroup of the nonlocal multiplier sums
constexpr int MAXQ = 27;

enum Mode { MODE_STEP = 0, MODE_FIELDS = 1, MODE_DIAG = 2, MODE_RECORD = 3 };

// Models: 0 conservative AC, 1 CH, 2 nonlocal / hybrid AC, 3 Liang2018,
// 4 Liang2014 with its hydrodynamics. The CH phase field (1, 4) stores the
// rest population of D3Q7 (its equilibrium is not zero there); the others
// give it weight 0 and do not store it.
__host__ __device__ constexpr int rest_offset(int model, bool d3) {
    return (model != 1 && model != 4 && d3) ? 1 : 0;
}

// physical constants, precomputed on the host (float64, and rounded once to
// float32 for the float32 forms)
template <class T>
struct PhysT {
    T rhoL, dRho;      // rho = rhoL + phi dRho (phi_H = 1, phi_L = 0)
    T muL, dMu;        // linear-mu interpolation of rho_X nu_X
    T nuL, dNu;        // linear-nu interpolation
    int visc_mu;       // 1: linear mu, 0: linear nu
    T beta4;           // 4 beta = 48 sigma / W
    T kappa;           // 3 sigma W / 2
    T anti;            // sqrt(2 beta / kappa) = 4 / W
    T eps2;            // normal regularisation eps^2
    T inv_tau_phi;     // 1 / tau_phi
    T g_fac_phi;       // 1 - 1 / (2 tau_phi)
    T eta;             // CH mobility parameter
    T s_o;             // MRT rate of the non-stress moments
    T lam;             // nonlocal model: weight of the conservative flux
    T mob;             // mobility M (nonlocal source)
    T w32;             // 4 beta / kappa = 32 / W^2
    T body[3];         // gravity (F_b = rho body + force)
    T force[3];
};
using Phys = PhysT<double>;

template <class T>
__host__ __device__ inline PhysT<float> to_float(const PhysT<T>& d) {
    PhysT<float> f;
    f.rhoL = (float)d.rhoL; f.dRho = (float)d.dRho;
    f.muL = (float)d.muL; f.dMu = (float)d.dMu;
    f.nuL = (float)d.nuL; f.dNu = (float)d.dNu;
    f.visc_mu = d.visc_mu;
    f.beta4 = (float)d.beta4; f.kappa = (float)d.kappa; f.anti = (float)d.anti;
    f.eps2 = (float)d.eps2; f.inv_tau_phi = (float)d.inv_tau_phi; f.g_fac_phi = (float)d.g_fac_phi;
    f.eta = (float)d.eta; f.s_o = (float)d.s_o;
    f.lam = (float)d.lam; f.mob = (float)d.mob; f.w32 = (float)d.w32;
    for (int k = 0; k < 3; ++k) { f.body[k] = (float)d.body[k]; f.force[k] = (float)d.force[k]; }
    return f;
}

// Device layout of every population array: plane-major [z][q][y][x], each
// population plane padded to P elements, so plane z of an array with Q
// populations starts at element z * Q * P.
//
// Streaming is a pull between two buffers per distribution: a buffer holds the
// post-collision populations of the previous step at their own node, slot i.
// The step loads population i of node x from node x - c_i (a node beyond a
// wall gives the bounce-back of slot opp(i) of x itself) and stores its
// post-collision populations at x in the other buffer, so every store is
// aligned to the node and only loads are shifted.
struct KArgs {
    const void* gin;       // hydrodynamic populations read this step [z][Qg][P]
    void* gout;            // hydrodynamic populations written this step [z][Qg][P]
    const void* hin;       // phase-field populations read this step [z][Qhs][P]
    void* hout;            // phase-field populations written this step [z][Qhs][P]
    void* phiu;            // CH / Liang: (phi u) of the previous step [z][3][P], compute type
    double* f_phi;         // MODE_FIELDS outputs (canonical float64), may be null
    double* f_u;
    double* f_p;
    double* f_rho;
    void* xg;              // MODE_RECORD: the state the step starts from, canonical
    void* xh;              //   g [Qg][nodes] and h [Qh][nodes], float64 (float32 if xf32)
    void* xpu;             //   and (phi u) [3][nodes] of the CH and Liang models, may be null
    int xf32;
    double* partials;      // MODE_DIAG per-block partials [nblocks][NDIAG]
    const double* gamma;   // nonlocal model: multiplier of this step (device)
    int P;                 // elements per population plane (>= nx * ny)
    int nx, ny, nz;
    int ntx, nty, ntz, zb; // tiles per axis, z planes per tile
    int tile;              // tile index (TILE_NX / TILE_NY), 3-D step only
    unsigned step;         // steps completed before this one (key of the stochastic rounding)
    int bc[3];             // 0 periodic, 1 wall
    int wall_axis;         // -1 none, else 0/1/2
    int write_h;           // 0 when phi is frozen
    int has_centre;
    double centre[3];
    double r_in, r_out;    // pressure regions r < r_in, r > r_out
    double gcorr[2][MAXQ]; // moving-wall term of a g population leaving through the low/high wall
    float gcorrf[2][MAXQ];
    Phys ph;
    PhysT<float> phf;
};

struct InitArgs {
    void* g;               // the buffers the first step reads
    void* h;
    void* phiu;
    const double* phi0;
    const double* u0;      // may be null
    const double* p0;      // may be null
    int P;
    int nx, ny, nz;
    int bc[3];
    double gcorr[2][MAXQ]; // moving-wall terms (see KArgs)
    Phys ph;
};

struct IOArgs {
    void* g;               // current hydrodynamic buffer (post-collision, unstreamed)
    void* h;               // current phase-field buffer
    double* cg;            // canonical float64 g [Qg][nodes] (post-streaming)
    double* ch;            // canonical float64 h [Qh][nodes]
    float* cgf;            // or, when set, canonical float32 g and h (read-out only)
    float* chf;
    int P;
    int nx, ny, nz;
    int bc[3];
    int wall_axis;
    double gcorr[2][MAXQ];
};

// float64 sums of the nonlocal multiplier over the current phase-field buffer
struct GammaArgs {
    const void* h;         // current (post-collision) phase-field buffer
    double* partials;      // [blocks][2]
    double* gamma;         // result
    int P;
    int nx, ny, nz;
    int bc[3];
    double w32;            // 4 beta / kappa
};

// discrete adjoint of one step on canonical arrays [q][z][y][x]: float64 for
// every model; float32 (R = float) for the AC model, its parameter partial
// sums still float64
template <class R>
struct AdjArgsT {
    const R* fg;           // forward state X^n (post-streaming)
    const R* fh;
    const R* lg;           // lambda^{n+1}
    const R* lh;
    R* og;                 // lambda^n (must not alias lg / lh)
    R* oh;
    const R* fpu;          // CH, Liang: (phi u) of the step before X^n [3][nodes]
    const R* lpu;          // its adjoint lambda_pu^{n+1}
    R* opu;                // lambda_pu^n
    R* dphi0;              // adjoint of the initialisation: dL/dphi0 (stencil pass, init mode)
    double* phi;           // workspace [nodes]: phi of the forward state, float64 in both forms
    R* work;               // workspace [5..9][nodes]
    double* partials;      // workspace [blocks][3]
    double* nlpart;        // nonlocal model: workspace [blocks][4] of partial sums
    double* nls;           // nonlocal model: workspace [4]: gamma, its denominator, dL/dgamma
    double* dparams;       // if set, the stencil pass adds the sum of the partials into it
    int nx, ny, nz;
    int bc[3];
    int qh;
    double sigma, W;
    Phys ph;
};
using AdjArgs = AdjArgsT<double>;

template <class R>
struct AdjInitArgsT {
    const R* lg;
    const R* lh;
    const R* lpu;          // Liang2018: lambda of (phi u) [3][nodes]
    const double* phi0;
    const double* u0;      // may be null
    const double* p0;      // may be null
    R* dphi0;
    int nx, ny, nz;
    Phys ph;
};
using AdjInitArgs = AdjInitArgsT<double>;

// launchers (kernels.hip, adjoint.hip); return hipSuccess or the launch error
hipError_t adjoint_scratch(int device, void** out);
hipError_t launch_adjoint_seed(const double* dphi, double* lg, double* lh, long long nn, int qg, int qh,
                               hipStream_t st);
hipError_t launch_adjoint(int lattice, int model, const AdjArgs& a, double* dparams, hipStream_t s);
hipError_t launch_adjoint_init(int lattice, int model, const AdjInitArgs& a, hipStream_t s);
hipError_t launch_adjoint_f32(int lattice, int model, const AdjArgsT<float>& a, double* dparams, hipStream_t s);
hipError_t launch_adjoint_init_ch_f32(int lattice, const AdjArgsT<float>& a, const double* phi0, const double* u0,
                                      const double* p0, double* dparams, hipStream_t s);
hipError_t launch_adjoint_seed_f32(const float* dphi, float* lg, float* lh, long long nn, int qg, int qh,
                                   hipStream_t s);
hipError_t launch_adjoint_init_f32(int lattice, const AdjInitArgsT<float>& a, hipStream_t s);
hipError_t launch_adjoint_seed_nl(int lattice, const AdjArgs& a, const double* dphi, double* lam_g, double* lam_h,
                                  double* dparams, hipStream_t s);
hipError_t launch_adjoint_init_ch(int lattice, int model, const AdjArgs& a, const double* phi0, const double* u0,
                                  const double* p0, double* dparams, hipStream_t s);
hipError_t launch_phiu_io(int precision, bool get, void* pu, double* canon, int P, int nx, int ny, int nz,
                          hipStream_t s);
hipError_t launch_step(int lattice, int model, int precision, int mode, const KArgs& a, hipStream_t s);
// per lattice pair (p) and model (m) instantiations (step_inst.hip)
hipError_t launch_step_p0_m0(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p0_m1(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p0_m2(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p1_m0(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p1_m1(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p1_m2(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p2_m0(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p2_m1(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p2_m2(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p0_m3(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p1_m3(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p2_m3(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p0_m4(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p1_m4(int precision, int mode, const KArgs& a, hipStream_t s);
hipError_t launch_step_p2_m4(int precision, int mode, const KArgs& a, hipStream_t s);
// resident workgroups per compute unit of the 3-D step kernel (0 if unknown)
int occupancy_step(int lattice, int model, int precision, int tile, int walls);
int occupancy_step_p0_m0(int precision, int tile, int walls);
int occupancy_step_p0_m1(int precision, int tile, int walls);
int occupancy_step_p0_m2(int precision, int tile, int walls);
int occupancy_step_p0_m3(int precision, int tile, int walls);
int occupancy_step_p0_m4(int precision, int tile, int walls);
int occupancy_step_p1_m0(int precision, int tile, int walls);
int occupancy_step_p1_m1(int precision, int tile, int walls);
int occupancy_step_p1_m2(int precision, int tile, int walls);
int occupancy_step_p1_m3(int precision, int tile, int walls);
int occupancy_step_p1_m4(int precision, int tile, int walls);
int occupancy_step_p2_m0(int precision, int tile, int walls);
int occupancy_step_p2_m1(int precision, int tile, int walls);
int occupancy_step_p2_m2(int precision, int tile, int walls);
int occupancy_step_p2_m3(int precision, int tile, int walls);
int occupancy_step_p2_m4(int precision, int tile, int walls);
hipError_t launch_init(int lattice, int model, int precision, const InitArgs& a, hipStream_t s);
hipError_t launch_get(int lattice, int model, int precision, const IOArgs& a, hipStream_t s);
hipError_t launch_set(int lattice, int model, int precision, const IOArgs& a, hipStream_t s);
hipError_t launch_reduce(const double* partials, int nblocks, double* out, hipStream_t s);
hipError_t launch_gamma(int lattice, int precision, const GammaArgs& a, hipStream_t s);
// checkpoint header (the first 256 bytes of a checkpoint): tag, step counter,
// checkpoint size and the layout it was written with (lattice, model,
// precision, nx, ny, nz), compared on the host before a load copies anything
struct CkHeader {
    static constexpr int N = 8;
    long long v[N];
};
hipError_t launch_header(void* dst, const CkHeader& hd, hipStream_t s);

}  // namespace pfk
