// C ABI of libpflbm (declared in include/pflbm.h): validation, device-state
// layout inside the caller's buffer, double-buffer bookkeeping and kernel
// launch orchestration. All arithmetic of the method runs in the
// kernels (kernels.hip); this file only sets up their arguments.
#include "pflbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.h"
#include "lattice.h"

using namespace pfk;

namespace {

struct Layout {
    int dim = 0, Qg = 0, Qh = 0, Qhs = 0;
    size_t sg = 0, sh = 0, sT = 0;   // bytes per stored g, h, compute value
    long long nodes = 0;
    int P = 0;                       // elements per population plane
    int ntx = 0, nty = 0, ntz = 0, zb = 0, nblocks = 0;   // 64 x 4 tiles (fields, diagnostics)
    int tile_step = 0, ntx_step = 0, nty_step = 0;        // tiles of the step kernel
    int zb_step = 0, ntz_step = 0;                        // z blocks of the step kernel
    size_t off_g[2] = {0, 0}, off_h[2] = {0, 0}, off_pu = 0, off_part = 0, off_gpart = 0, off_res = 0,
           total = 0;
    size_t ck_g = 0, ck_h = 0, ck_pu = 0, ck_total = 0;
    size_t g_bytes = 0, h_bytes = 0, pu_bytes = 0;
};

constexpr size_t ALIGN = 4096;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool finite(double v) { return std::isfinite(v); }

// validate; returns an error message or empty string
std::string validate(const pflbm_params& p) {
    if (p.lattice != PFLBM_D2Q9_D2Q5 && p.lattice != PFLBM_D3Q19_D3Q7 && p.lattice != PFLBM_D3Q27_D3Q7)
        return "lattice must be PFLBM_D2Q9_D2Q5, PFLBM_D3Q19_D3Q7 or PFLBM_D3Q27_D3Q7";
    if (p.model != PFLBM_AC && p.model != PFLBM_CH && p.model != PFLBM_NL && p.model != PFLBM_L18 &&
        p.model != PFLBM_L14)
        return "model must be PFLBM_AC, PFLBM_CH, PFLBM_NL, PFLBM_L18 or PFLBM_L14";
    if (p.precision < PFLBM_FP64 || p.precision > PFLBM_MIXED_BF16) return "unknown precision";
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return "nx, ny, nz must be >= 1";
    if (p.lattice == PFLBM_D2Q9_D2Q5 && p.nz != 1) return "2-D lattice requires nz == 1";
    const long long nodes = (long long)p.nx * p.ny * p.nz;
    if (nodes > 0x7fffffffLL) return "more than 2^31-1 nodes";
    if ((long long)p.nx * p.ny > 0x7fff0000LL) return "more than 2^31 nodes per z plane";
    {
        // kernels address a population plane as a scalar base plus a 32-bit
        // byte offset: one plane (padded to 64 nodes) must stay below 4 GiB
        const long long esz = p.precision == PFLBM_FP64 ? 8 : 4;
        const long long padded = ((long long)p.nx * p.ny + 63) / 64 * 64;
        if (padded * esz > 0xffffffffLL) return "one z plane of a population spans 4 GiB or more";
    }
    int walls = 0;
    for (int a = 0; a < 3; ++a) {
        if (p.bc[a] != PFLBM_PERIODIC && p.bc[a] != PFLBM_WALL) return "bc must be PFLBM_PERIODIC or PFLBM_WALL";
        walls += p.bc[a] == PFLBM_WALL;
    }
    if (walls > 1) return "walls on more than one axis are not supported";
    if (p.lattice == PFLBM_D2Q9_D2Q5 && p.bc[2] != PFLBM_PERIODIC) return "2-D lattice requires a periodic z axis";
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 3; ++a) {
            if (!finite(p.wall_u[s][a])) return "wall velocity not finite";
            if (p.bc[a] == PFLBM_WALL && p.wall_u[s][a] != 0.0) return "wall velocity must be tangential to the wall";
            if (p.lattice == PFLBM_D2Q9_D2Q5 && a == 2 && p.wall_u[s][a] != 0.0) return "2-D wall velocity has a z component";
        }
    if (!(p.rho_H > 0) || !(p.rho_L > 0) || !finite(p.rho_H) || !finite(p.rho_L)) return "rho_H and rho_L must be > 0";
    if (!(p.nu_H > 0) || !(p.nu_L > 0) || !finite(p.nu_H) || !finite(p.nu_L)) return "nu_H and nu_L must be > 0 (tau > 1/2)";
    if (p.visc_interp != PFLBM_VISC_LINEAR_MU && p.visc_interp != PFLBM_VISC_LINEAR_NU) return "unknown viscosity interpolation";
    if (!(p.M > 0) || !finite(p.M)) return "M must be > 0";
    if (!(p.W > 0) || !finite(p.W)) return "W must be > 0";
    if (!(p.sigma >= 0) || !finite(p.sigma)) return "sigma must be >= 0";
    if (!(p.eta > 0) || !finite(p.eta)) return "eta must be > 0";
    if (!(p.s_other > 0 && p.s_other < 2)) return "s_other must be in (0, 2)";
    if (!(p.normal_eps >= 0) || !finite(p.normal_eps)) return "normal_eps must be >= 0";
    if (!(p.lam >= 0 && p.lam <= 1)) return "lam must be in [0, 1]";
    if (p.model == PFLBM_L18 || p.model == PFLBM_L14) {
        for (int s = 0; s < 2; ++s)
            for (int a = 0; a < 3; ++a)
                if (p.wall_u[s][a] != 0.0) return "the Liang models support stationary walls only";
        if (p.precision == PFLBM_MIXED_FP16 && (p.rho_H > 16.0 || p.rho_L > 16.0))
            return "the Liang models with fp16-stored g need rho_H, rho_L <= 16";
    }
    for (int a = 0; a < 3; ++a)
        if (!finite(p.gravity[a]) || !finite(p.force[a])) return "body force not finite";
    if (p.lattice == PFLBM_D2Q9_D2Q5 && (p.gravity[2] != 0.0 || p.force[2] != 0.0)) return "2-D body force has a z component";
    if (p.check_interval < 0) return "check_interval must be >= 0";
    if (p.zblock < 0) return "zblock must be >= 0";
    if (p.tile < PFLBM_TILE_AUTO || p.tile > PFLBM_TILE_128x8) return "unknown tile";
    return "";
}

Layout make_layout(const pflbm_params& p) {
    Layout L;
    const bool d3 = p.lattice != PFLBM_D2Q9_D2Q5;
    L.dim = d3 ? 3 : 2;
    L.Qg = p.lattice == PFLBM_D3Q27_D3Q7 ? 27 : (d3 ? 19 : 9);
    L.Qh = d3 ? 7 : 5;
    L.Qhs = rest_offset(p.model, d3) ? 6 : L.Qh;   // D3Q7 rest population of weight 0 not stored
    L.sT = p.precision == PFLBM_FP64 ? 8 : 4;
    L.sg = p.precision == PFLBM_FP64 ? 8 : (p.precision == PFLBM_FP32 ? 4 : 2);
    L.sh = p.precision == PFLBM_FP64 ? 8 : 4;
    L.nodes = (long long)p.nx * p.ny * p.nz;
    L.P = (int)align_up((size_t)p.nx * p.ny, 64);
    const size_t planes = (size_t)p.nz * L.P;
    L.ntx = (p.nx + TILE_NX[0] - 1) / TILE_NX[0];
    L.nty = (p.ny + TILE_NY[0] - 1) / TILE_NY[0];
    // step tile: measured fastest per storage form on the 256^3 droplet case;
    // no wider than nx needs. 256 x 4 (1024 threads, XCD runs) allows 128
    // registers per thread: the float32 and fp16 / bf16-stored kernels fit
    // (90-128) except Liang2014 on D3Q27, whose 16-bit form runs faster in
    // 64 x 4; float64 needs 168-227 and takes 128 x 2. Liang2014 with 16-bit
    // g on D3Q19 takes 128 x 8: its phi frame reaches two nodes out, and the
    // taller tile has a quarter less frame per node (6 % faster).
    int t = 0;
    if (d3) {
        const bool half = p.precision == PFLBM_MIXED_FP16 || p.precision == PFLBM_MIXED_BF16;
        const bool fits = !(p.model == PFLBM_L14 && p.lattice == PFLBM_D3Q27_D3Q7 && half);
        if (p.tile != PFLBM_TILE_AUTO) t = p.tile - PFLBM_TILE_64x4;
        else if (p.precision == PFLBM_FP64) t = p.nx > 64 ? 1 : 0;
        else if (half && p.model == PFLBM_L14 && p.lattice == PFLBM_D3Q19_D3Q7 && p.nx >= 128) t = 4;
        else if (p.nx >= 256 && fits) t = 3;
        else if (p.precision == PFLBM_FP32 && fits) t = p.nx > 64 ? 1 : 0;
    }
    L.tile_step = t;
    L.ntx_step = (p.nx + TILE_NX[t] - 1) / TILE_NX[t];
    L.nty_step = (p.ny + TILE_NY[t] - 1) / TILE_NY[t];
    if (d3) {
        L.zb = p.zblock > 0 ? p.zblock : 8;
        if (L.zb > p.nz) L.zb = p.nz;
    } else {
        L.zb = 1;
    }
    L.ntz = (p.nz + L.zb - 1) / L.zb;
    L.nblocks = L.ntx * L.nty * L.ntz;
    L.zb_step = L.zb;   // refined at create time when zblock is automatic
    L.ntz_step = L.ntz;
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
        L.off_g[k] = off;
        off = align_up(off + (size_t)L.Qg * planes * L.sg, ALIGN);
    }
    for (int k = 0; k < 2; ++k) {
        L.off_h[k] = off;
        off = align_up(off + (size_t)L.Qhs * planes * L.sh, ALIGN);
    }
    L.off_pu = off;
    const bool has_pu = p.model == PFLBM_CH || p.model == PFLBM_L18 || p.model == PFLBM_L14;
    if (has_pu) off = align_up(off + 3 * planes * L.sT, ALIGN);
    L.off_part = off;
    off = align_up(off + (size_t)L.nblocks * NDIAG * sizeof(double), ALIGN);
    L.off_gpart = off;   // nonlocal multiplier: per-256-node partial sums
    if (p.model == PFLBM_NL) {
        const size_t nbg = (size_t)((p.nx * p.ny + 255) / 256) * ((p.nz + GAMMA_ZB - 1) / GAMMA_ZB);
        off = align_up(off + nbg * 2 * sizeof(double), ALIGN);
    }
    L.off_res = off;
    off = align_up(off + 64 * sizeof(double), ALIGN);
    L.total = off;
    // checkpoint: 256-byte header, current g, current h, (phi u)
    L.ck_g = 256;
    L.g_bytes = (size_t)L.Qg * planes * L.sg;
    L.h_bytes = (size_t)L.Qhs * planes * L.sh;
    L.pu_bytes = has_pu ? 3 * planes * L.sT : 0;
    L.ck_h = align_up(L.ck_g + L.g_bytes, 256);
    L.ck_pu = align_up(L.ck_h + L.h_bytes, 256);
    L.ck_total = align_up(L.ck_pu + L.pu_bytes, 256);
    return L;
}

template <class GL>
void wall_terms(const pflbm_params& p, double gcorr[2][MAXQ]) {
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < MAXQ; ++i) gcorr[s][i] = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < GL::Q; ++i) {
            // population i leaving through wall s: -2 w_i (c_i . u_w) / c_s^2
            const double cu = GL::c(i, 0) * p.wall_u[s][0] + GL::c(i, 1) * p.wall_u[s][1] +
                              GL::c(i, 2) * p.wall_u[s][2];
            gcorr[s][i] = -6.0 * GL::w(i) * cu;
        }
}

}  // namespace

struct pflbm {
    pflbm_params p;
    Layout L;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    int device = 0;
    int gcur = 0, hcur = 0;   // buffers the next step reads
    long long steps = 0;
    bool initialised = false;
    int sticky = 0;        // PFLBM_EHIP: every later call returns PFLBM_ESTATE
    bool unstable = false; // after PFLBM_EUNSTABLE, until pflbm_init / pflbm_load_state
    std::string err;
    Phys ph;
    PhysT<float> phf;
    double gcorr[2][MAXQ];
    float gcorrf[2][MAXQ];
    int wall_axis = -1;
    double res_host[NDIAG];
};

namespace {

int fail(pflbm_t* h, int code, const std::string& msg) {
    if (h) {
        h->err = msg;
        // a rejected call (EINVAL, EUNSUPPORTED) leaves the handle as it was
        if (code == PFLBM_EUNSTABLE) h->unstable = true;
        else if (code == PFLBM_EHIP) h->sticky = code;
    }
    return code;
}

int hip_fail(pflbm_t* h, hipError_t e, const char* where) {
    return fail(h, PFLBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call, where)                       \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(h, e_, where); \
    } while (0)

int guard(pflbm_t* h) {
    if (!h) return PFLBM_EINVAL;
    if (h->sticky || h->unstable) return PFLBM_ESTATE;
    return PFLBM_OK;
}

// calls that replace the whole state (init, load_state) are allowed after an
// instability and clear it when they succeed
int guard_replace(pflbm_t* h) {
    if (!h) return PFLBM_EINVAL;
    if (h->sticky) return PFLBM_ESTATE;
    return PFLBM_OK;
}

// z planes per workgroup of a z-marching pass when the caller leaves zblock
// at 0, from its tile and resident workgroups per compute unit. A workgroup
// marches its column plane by plane and first loads the halo planes of its
// phi ring; with one resident workgroup per compute unit (the 1024-thread
// tile) nothing hides that start, so the grid is sized to fill every unit
// once. With several resident workgroups: 32 planes while that still leaves
// two rounds of work, else halving down to 8. Returns 0 if the device cannot
// be queried (the layout's depth stays).
int auto_zblock(const pflbm_t* h, int tile, int occ) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) return 0;
    if (cus <= 0 || occ <= 0) return 0;
    const long long slots = (long long)cus * occ;
    const long long tiles = (long long)((h->p.nx + TILE_NX[tile] - 1) / TILE_NX[tile]) *
                            ((h->p.ny + TILE_NY[tile] - 1) / TILE_NY[tile]);
    const int nz = h->p.nz;
    int zb;
    if (occ == 1) {
        const long long nzb = slots / tiles > 1 ? slots / tiles : 1;
        zb = (int)((nz + nzb - 1) / nzb);
        if (zb < 4) zb = 4;
    } else {
        zb = 32;
        while (zb > 8 && tiles * ((nz + zb - 1) / zb) < 2 * slots) zb /= 2;
    }
    return zb > nz ? nz : zb;
}

// the step kernel's depth; the fields and diagnostics kernels keep the layout's
// depth (their partial sums are sized by it)
void choose_zblocks(pflbm_t* h) {
    Layout& L = h->L;
    if (L.dim != 3 || h->p.zblock != 0 || h->device < 0) return;
    const int walls = h->wall_axis >= 0;
    const int zb = auto_zblock(h, L.tile_step,
                               occupancy_step(h->p.lattice, h->p.model, h->p.precision, L.tile_step, walls));
    if (zb > 0) {
        L.zb_step = zb;
        L.ntz_step = (h->p.nz + zb - 1) / zb;
    }
}

void base_args(pflbm_t* h, KArgs& a) {
    std::memset(&a, 0, sizeof(a));
    a.gin = h->base + h->L.off_g[h->gcur];
    a.gout = h->base + h->L.off_g[1 - h->gcur];
    a.hin = h->base + h->L.off_h[h->hcur];
    a.hout = h->base + h->L.off_h[1 - h->hcur];
    a.phiu = h->base + h->L.off_pu;
    a.partials = (double*)(h->base + h->L.off_part);
    a.P = h->L.P;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    a.ntx = h->L.ntx;
    a.nty = h->L.nty;
    a.ntz = h->L.ntz;
    a.zb = h->L.zb;
    for (int k = 0; k < 3; ++k) a.bc[k] = h->p.bc[k];
    a.wall_axis = h->wall_axis;
    a.write_h = h->p.freeze_phi ? 0 : 1;
    std::memcpy(a.gcorr, h->gcorr, sizeof(a.gcorr));
    std::memcpy(a.gcorrf, h->gcorrf, sizeof(a.gcorrf));
    a.ph = h->ph;
    a.phf = h->phf;
}

// nonlocal model: the multiplier of the current state into its device slot
constexpr int RES_GAMMA = 32;   // index in the result area

int run_gamma(pflbm_t* h, KArgs& a) {
    if (h->p.model != PFLBM_NL) return PFLBM_OK;
    GammaArgs ga;
    std::memset(&ga, 0, sizeof(ga));
    ga.h = h->base + h->L.off_h[h->hcur];
    ga.partials = (double*)(h->base + h->L.off_gpart);
    ga.gamma = (double*)(h->base + h->L.off_res) + RES_GAMMA;
    ga.P = h->L.P;
    ga.nx = h->p.nx;
    ga.ny = h->p.ny;
    ga.nz = h->p.nz;
    for (int k = 0; k < 3; ++k) ga.bc[k] = h->p.bc[k];
    ga.w32 = h->ph.w32;
    HIPCHK(h, launch_gamma(h->p.lattice, h->p.precision, ga, h->stream), "nonlocal multiplier kernels");
    a.gamma = ga.gamma;
    return PFLBM_OK;
}

int run_diag(pflbm_t* h, const double* centre, double R, double* res) {
    KArgs a;
    base_args(h, a);
    if (int st = run_gamma(h, a)) return st;
    if (centre) {
        a.has_centre = 1;
        for (int k = 0; k < h->L.dim; ++k) a.centre[k] = centre[k];
        a.r_in = R - 2.0 * h->p.W;
        a.r_out = R + 2.0 * h->p.W;
    }
    HIPCHK(h, launch_step(h->p.lattice, h->p.model, h->p.precision, MODE_DIAG, a, h->stream), "diag kernel");
    double* dres = (double*)(h->base + h->L.off_res);
    HIPCHK(h, launch_reduce(a.partials, h->L.nblocks, dres, h->stream), "reduce kernel");
    HIPCHK(h, hipMemcpyAsync(res, dres, NDIAG * sizeof(double), hipMemcpyDeviceToHost, h->stream), "diag copy");
    HIPCHK(h, hipStreamSynchronize(h->stream), "diag sync");
    return PFLBM_OK;
}

}  // namespace

extern "C" {

const char* pflbm_strerror(int status) {
    switch (status) {
        case PFLBM_OK: return "ok";
        case PFLBM_EINVAL: return "invalid argument";
        case PFLBM_EUNSUPPORTED: return "unsupported";
        case PFLBM_EHIP: return "HIP runtime error";
        case PFLBM_EUNSTABLE: return "numerical instability (NaN/Inf or rho <= 0)";
        case PFLBM_ESTATE: return "handle in error state";
        default: return "unknown status";
    }
}

int pflbm_state_bytes(const pflbm_params* params, size_t* bytes) {
    if (!params || !bytes) return PFLBM_EINVAL;
    if (!validate(*params).empty()) return PFLBM_EINVAL;
    *bytes = make_layout(*params).total;
    return PFLBM_OK;
}

int pflbm_create(const pflbm_params* params, void* hip_stream, void* dev_state, size_t bytes,
                 pflbm_t** out) {
    if (!params || !out) return PFLBM_EINVAL;
    *out = nullptr;
    if (!validate(*params).empty()) return PFLBM_EINVAL;
    const Layout L = make_layout(*params);
    if (!dev_state || bytes < L.total || ((uintptr_t)dev_state % 256) != 0) return PFLBM_EINVAL;
    pflbm_t* h = new (std::nothrow) pflbm();
    if (!h) return PFLBM_EINVAL;
    h->p = *params;
    h->L = L;
    h->stream = (hipStream_t)hip_stream;
    h->base = (char*)dev_state;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    const pflbm_params& p = h->p;
    for (int a = 0; a < 3; ++a)
        if (p.bc[a] == PFLBM_WALL) h->wall_axis = a;
    choose_zblocks(h);
    if (p.lattice == PFLBM_D2Q9_D2Q5) wall_terms<D2Q9>(p, h->gcorr);
    else if (p.lattice == PFLBM_D3Q19_D3Q7) wall_terms<D3Q19>(p, h->gcorr);
    else wall_terms<D3Q27>(p, h->gcorr);
    Phys& ph = h->ph;
    ph.rhoL = p.rho_L;
    ph.dRho = p.rho_H - p.rho_L;
    ph.muL = p.rho_L * p.nu_L;
    ph.dMu = p.rho_H * p.nu_H - p.rho_L * p.nu_L;
    ph.nuL = p.nu_L;
    ph.dNu = p.nu_H - p.nu_L;
    ph.visc_mu = p.visc_interp == PFLBM_VISC_LINEAR_MU;
    ph.beta4 = 4.0 * 12.0 * p.sigma / p.W;   // 4 beta, beta = 12 sigma / W
    ph.kappa = 1.5 * p.sigma * p.W;          // kappa = 3 sigma W / 2
    ph.anti = 4.0 / p.W;                     // sqrt(2 beta / kappa)
    ph.eps2 = p.normal_eps * p.normal_eps;
    const bool ch_phase = p.model == PFLBM_CH || p.model == PFLBM_L14;
    const double tau_phi = ch_phase ? 3.0 * p.M / p.eta + 0.5 : 3.0 * p.M + 0.5;
    ph.inv_tau_phi = 1.0 / tau_phi;
    ph.g_fac_phi = 1.0 - 0.5 / tau_phi;
    ph.eta = p.eta;
    ph.s_o = p.s_other;
    ph.lam = p.lam;
    ph.mob = p.M;
    ph.w32 = 32.0 / (p.W * p.W);              // 4 beta / kappa
    for (int a = 0; a < 3; ++a) {
        ph.body[a] = p.gravity[a];
        ph.force[a] = p.force[a];
    }
    h->phf = to_float(ph);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < MAXQ; ++i) h->gcorrf[s][i] = (float)h->gcorr[s][i];
    *out = h;
    return PFLBM_OK;
}

void pflbm_destroy(pflbm_t* h) { delete h; }

const char* pflbm_last_error(const pflbm_t* h) { return h ? h->err.c_str() : "null handle"; }

int pflbm_init(pflbm_t* h, const double* phi0, const double* u0, const double* p0) {
    int st = guard_replace(h);
    if (st) return st;
    if (!phi0) return fail(h, PFLBM_EINVAL, "phi0 is null");
    InitArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = h->base + h->L.off_g[0];
    a.h = h->base + h->L.off_h[0];
    a.phiu = h->base + h->L.off_pu;
    a.phi0 = phi0;
    a.u0 = u0;
    a.p0 = p0;
    a.P = h->L.P;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    for (int k = 0; k < 3; ++k) a.bc[k] = h->p.bc[k];
    std::memcpy(a.gcorr, h->gcorr, sizeof(a.gcorr));
    a.ph = h->ph;
    HIPCHK(h, launch_init(h->p.lattice, h->p.model, h->p.precision, a, h->stream), "init kernel");
    h->gcur = 0;
    h->hcur = 0;
    h->steps = 0;
    h->initialised = true;
    h->unstable = false;
    return PFLBM_OK;
}

// one step from the current buffers into the other ones; the tile, grid and
// recording outputs are the caller's (a)
static int step_once(pflbm_t* h, KArgs& a, int mode) {
    a.gin = h->base + h->L.off_g[h->gcur];
    a.gout = h->base + h->L.off_g[1 - h->gcur];
    a.hin = h->base + h->L.off_h[h->hcur];
    a.hout = h->base + h->L.off_h[1 - h->hcur];
    a.step = (unsigned)h->steps;
    if (int st = run_gamma(h, a)) return st;
    HIPCHK(h, launch_step(h->p.lattice, h->p.model, h->p.precision, mode, a, h->stream), "step kernel");
    if (!h->p.freeze_phi) h->hcur ^= 1;
    h->gcur ^= 1;
    h->steps += 1;
    if (h->p.check_interval > 0 && h->steps % h->p.check_interval == 0) {
        if (int st = run_diag(h, nullptr, 0.0, h->res_host)) return st;
        if (h->res_host[10] > 0.0) {
            char buf[128];
            std::snprintf(buf, sizeof(buf), "NaN/Inf or rho <= 0 detected after step %lld", h->steps);
            return fail(h, PFLBM_EUNSTABLE, buf);
        }
    }
    return PFLBM_OK;
}

int pflbm_step(pflbm_t* h, int nsteps) {
    int st = guard(h);
    if (st) return st;
    if (nsteps < 0) return fail(h, PFLBM_EINVAL, "nsteps < 0");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    KArgs a;
    base_args(h, a);
    a.tile = h->L.tile_step;
    a.ntx = h->L.ntx_step;
    a.nty = h->L.nty_step;
    a.ntz = h->L.ntz_step;
    a.zb = h->L.zb_step;
    for (int k = 0; k < nsteps; ++k)
        if ((st = step_once(h, a, MODE_STEP))) return st;
    return PFLBM_OK;
}

// one step that also writes the state it starts from (canonical layout)
static int step_record(pflbm_t* h, void* g, void* hd, void* pu, int f32) {
    int st = guard(h);
    if (st) return st;
    if (!g || !hd) return fail(h, PFLBM_EINVAL, "null output");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    if (h->p.precision != PFLBM_FP64 && h->p.precision != PFLBM_FP32)
        return fail(h, PFLBM_EUNSUPPORTED, "the recording step covers the float64 and float32 forms");
    KArgs a;
    base_args(h, a);
    a.xg = g;
    a.xh = hd;
    a.xpu = (h->p.model == PFLBM_CH || h->p.model == PFLBM_L18 || h->p.model == PFLBM_L14) ? pu : nullptr;
    a.xf32 = f32;
    // 128 x 2 tiles where the box is wide enough (64 x 4 otherwise), the
    // layout's z depth
    const int t = (h->L.dim == 3 && h->p.nx > 64) ? 1 : 0;
    a.tile = t;
    a.ntx = (h->p.nx + TILE_NX[t] - 1) / TILE_NX[t];
    a.nty = (h->p.ny + TILE_NY[t] - 1) / TILE_NY[t];
    a.zb = h->L.zb;
    a.ntz = (h->p.nz + a.zb - 1) / a.zb;
    return step_once(h, a, MODE_RECORD);
}

int pflbm_step_record(pflbm_t* h, double* g, double* hd, double* pu) { return step_record(h, g, hd, pu, 0); }

int pflbm_step_record_f32(pflbm_t* h, float* g, float* hd, float* pu) { return step_record(h, g, hd, pu, 1); }

int pflbm_fields(pflbm_t* h, double* phi, double* u, double* p, double* rho) {
    int st = guard(h);
    if (st) return st;
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    KArgs a;
    base_args(h, a);
    a.f_phi = phi;
    a.f_u = u;
    a.f_p = p;
    a.f_rho = rho;
    if ((st = run_gamma(h, a))) return st;
    HIPCHK(h, launch_step(h->p.lattice, h->p.model, h->p.precision, MODE_FIELDS, a, h->stream), "fields kernel");
    return PFLBM_OK;
}

int pflbm_volume(pflbm_t* h, const double* centre, double R, pflbm_diag* out) {
    int st = guard(h);
    if (st) return st;
    if (!out) return fail(h, PFLBM_EINVAL, "out is null");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    st = run_diag(h, centre, R, h->res_host);
    if (st) return st;
    const double* r = h->res_host;
    out->V_phi = r[0];
    out->V_count = r[1];
    out->sum_phi = r[2];
    out->phi_min = r[3];
    out->phi_max = r[4];
    out->umax = std::sqrt(r[5]);
    out->n_in = (long long)r[7];
    out->n_out = (long long)r[9];
    out->p_in = r[7] > 0 ? r[6] / r[7] : NAN;
    out->p_out = r[9] > 0 ? r[8] / r[9] : NAN;
    out->unstable = r[10] > 0.0 ? 1 : 0;
    return PFLBM_OK;
}

static void io_args(pflbm_t* h, IOArgs& a) {
    std::memset(&a, 0, sizeof(a));
    a.g = h->base + h->L.off_g[h->gcur];
    a.h = h->base + h->L.off_h[h->hcur];
    a.P = h->L.P;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    for (int k = 0; k < 3; ++k) a.bc[k] = h->p.bc[k];
    a.wall_axis = h->wall_axis;
    std::memcpy(a.gcorr, h->gcorr, sizeof(a.gcorr));
}

int pflbm_get_distributions(pflbm_t* h, double* g, double* hd) {
    int st = guard(h);
    if (st) return st;
    if (!g || !hd) return fail(h, PFLBM_EINVAL, "null output");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    IOArgs a;
    io_args(h, a);
    a.cg = g;
    a.ch = hd;
    HIPCHK(h, launch_get(h->p.lattice, h->p.model, h->p.precision, a, h->stream), "get kernel");
    return PFLBM_OK;
}

int pflbm_get_distributions_f32(pflbm_t* h, float* g, float* hd) {
    int st = guard(h);
    if (st) return st;
    if (!g || !hd) return fail(h, PFLBM_EINVAL, "null output");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    IOArgs a;
    io_args(h, a);
    a.cgf = g;
    a.chf = hd;
    HIPCHK(h, launch_get(h->p.lattice, h->p.model, h->p.precision, a, h->stream), "get kernel");
    return PFLBM_OK;
}

int pflbm_set_distributions(pflbm_t* h, const double* g, const double* hd) {
    int st = guard(h);
    if (st) return st;
    if (!g || !hd) return fail(h, PFLBM_EINVAL, "null input");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    IOArgs a;
    io_args(h, a);
    a.cg = (double*)g;
    a.ch = (double*)hd;
    HIPCHK(h, launch_set(h->p.lattice, h->p.model, h->p.precision, a, h->stream), "set kernel");
    return PFLBM_OK;
}

int pflbm_step_count(const pflbm_t* h, long long* steps) {
    if (!h || !steps) return PFLBM_EINVAL;
    *steps = h->steps;
    return PFLBM_OK;
}

static CkHeader ck_header(const pflbm_t* h, long long steps) {
    CkHeader hd;
    hd.v[0] = 0x70666c626eLL;   // tag (post-collision pull layout)
    hd.v[1] = steps;
    hd.v[2] = (long long)h->L.ck_total;
    hd.v[3] = h->p.lattice + 16LL * h->p.model + 256LL * h->p.precision + 4096LL * (h->p.freeze_phi != 0);
    hd.v[4] = h->p.nx;
    hd.v[5] = h->p.ny;
    hd.v[6] = h->p.nz;
    hd.v[7] = 0;
    return hd;
}

int pflbm_checkpoint_bytes(const pflbm_t* h, size_t* bytes) {
    if (!h || !bytes) return PFLBM_EINVAL;
    *bytes = h->L.ck_total;
    return PFLBM_OK;
}

int pflbm_save_state(pflbm_t* h, void* dev_dst) {
    int st = guard(h);
    if (st) return st;
    if (!dev_dst) return fail(h, PFLBM_EINVAL, "null destination");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    char* d = (char*)dev_dst;
    const Layout& L = h->L;
    HIPCHK(h, launch_header(d, ck_header(h, h->steps), h->stream), "header kernel");
    HIPCHK(h, hipMemcpyAsync(d + L.ck_g, h->base + L.off_g[h->gcur], L.g_bytes, hipMemcpyDeviceToDevice, h->stream), "save g");
    HIPCHK(h, hipMemcpyAsync(d + L.ck_h, h->base + L.off_h[h->hcur], L.h_bytes, hipMemcpyDeviceToDevice, h->stream), "save h");
    if (L.pu_bytes)
        HIPCHK(h, hipMemcpyAsync(d + L.ck_pu, h->base + L.off_pu, L.pu_bytes, hipMemcpyDeviceToDevice, h->stream), "save phiu");
    return PFLBM_OK;
}

int pflbm_load_state(pflbm_t* h, const void* dev_src) {
    int st = guard_replace(h);
    if (st) return st;
    if (!dev_src) return fail(h, PFLBM_EINVAL, "null source");
    const char* s = (const char*)dev_src;
    const Layout& L = h->L;
    CkHeader hdr;
    HIPCHK(h, hipMemcpyAsync(hdr.v, s, sizeof(hdr.v), hipMemcpyDeviceToHost, h->stream), "load header");
    HIPCHK(h, hipStreamSynchronize(h->stream), "load sync");
    const CkHeader want = ck_header(h, hdr.v[1]);
    if (hdr.v[0] != want.v[0]) return fail(h, PFLBM_EINVAL, "not a pflbm checkpoint");
    if (hdr.v[2] != want.v[2]) return fail(h, PFLBM_EINVAL, "checkpoint size differs from this handle's");
    for (int k = 3; k < CkHeader::N; ++k)
        if (hdr.v[k] != want.v[k])
            return fail(h, PFLBM_EINVAL, "checkpoint written with another lattice, model, precision or box");
    if (hdr.v[1] < 0) return fail(h, PFLBM_EINVAL, "checkpoint step counter is negative");
    HIPCHK(h, hipMemcpyAsync(h->base + L.off_g[0], s + L.ck_g, L.g_bytes, hipMemcpyDeviceToDevice, h->stream), "load g");
    HIPCHK(h, hipMemcpyAsync(h->base + L.off_h[0], s + L.ck_h, L.h_bytes, hipMemcpyDeviceToDevice, h->stream), "load h");
    if (L.pu_bytes)
        HIPCHK(h, hipMemcpyAsync(h->base + L.off_pu, s + L.ck_pu, L.pu_bytes, hipMemcpyDeviceToDevice, h->stream), "load phiu");
    h->steps = hdr.v[1];
    h->gcur = 0;
    h->hcur = 0;
    h->initialised = true;
    h->unstable = false;
    return PFLBM_OK;
}

static size_t adj_nodes(const pflbm_t* h) { return (size_t)h->p.nx * h->p.ny * h->p.nz; }

// per-node adjoint values of the workspace: dL/dphi, dL/dgrad phi, dL/dlap phi;
// the nonlocal model adds dL/dR and phi = sum h, Liang2014 mu_phi, lap phi,
// dL/dmu_phi and dL/dlap mu_phi
static size_t adj_nwork(const pflbm_t* h) {
    return h->p.model == PFLBM_NL ? 7 : (h->p.model == PFLBM_L14 ? 9 : 5);
}

int pflbm_adjoint_workspace_bytes(const pflbm_t* h, size_t* bytes) {
    if (!h || !bytes) return PFLBM_EINVAL;
    const size_t nn = adj_nodes(h);
    const size_t blocks = (nn + 255) / 256;
    size_t b = align_up(nn * 8, 256) + align_up(adj_nwork(h) * nn * 8, 256) + align_up(blocks * 3 * 8, 256);
    if (h->p.model == PFLBM_NL) b += align_up(blocks * 4 * 8, 256) + 256;
    *bytes = b;
    return PFLBM_OK;
}

// with_pu: the entry point carries the (phi u) state of the CH model
static int adjoint_check(pflbm_t* h, bool with_pu) {
    int st = guard(h);
    if (st) return st;
    const bool has_pu = h->p.model == PFLBM_CH || h->p.model == PFLBM_L18 || h->p.model == PFLBM_L14;
    if (has_pu && !with_pu)
        return fail(h, PFLBM_EUNSUPPORTED, "the CH and Liang adjoints carry (phi u): use the _pu entry points");
    if (h->p.freeze_phi) return fail(h, PFLBM_EUNSUPPORTED, "adjoint of a frozen phase field is not implemented");
    return PFLBM_OK;
}

static int adjoint_run(pflbm_t* h, const double* fwd_g, const double* fwd_h, const double* fwd_pu,
                       const double* lam_g, const double* lam_h, const double* lam_pu, double* lam_g_out,
                       double* lam_h_out, double* lam_pu_out, double* dparams, void* work);

int pflbm_adjoint_step(pflbm_t* h, const double* fwd_g, const double* fwd_h, const double* lam_g,
                       const double* lam_h, double* lam_g_out, double* lam_h_out, double* dparams,
                       void* work) {
    if (int st = adjoint_check(h, false)) return st;
    if (!work) return fail(h, PFLBM_EINVAL, "null pointer");
    return adjoint_run(h, fwd_g, fwd_h, nullptr, lam_g, lam_h, nullptr, lam_g_out, lam_h_out, nullptr, dparams,
                       work);
}

int pflbm_adjoint_step_pu(pflbm_t* h, const double* fwd_g, const double* fwd_h, const double* fwd_pu,
                          const double* lam_g, const double* lam_h, const double* lam_pu, double* lam_g_out,
                          double* lam_h_out, double* lam_pu_out, double* dparams, void* work) {
    if (int st = adjoint_check(h, true)) return st;
    if (!work) return fail(h, PFLBM_EINVAL, "null pointer");
    if (h->p.model != PFLBM_CH && h->p.model != PFLBM_L18 && h->p.model != PFLBM_L14) {
        fwd_pu = lam_pu = nullptr;
        lam_pu_out = nullptr;
    } else {
        if (!fwd_pu || !lam_pu || !lam_pu_out) return fail(h, PFLBM_EINVAL, "null pointer");
        if (lam_pu_out == lam_pu) return fail(h, PFLBM_EINVAL, "lambda in and out must not alias");
    }
    return adjoint_run(h, fwd_g, fwd_h, fwd_pu, lam_g, lam_h, lam_pu, lam_g_out, lam_h_out, lam_pu_out, dparams,
                       work);
}

int pflbm_adjoint_step_noalloc(pflbm_t* h, const double* fwd_g, const double* fwd_h, const double* lam_g,
                               const double* lam_h, double* lam_g_out, double* lam_h_out, double* dparams) {
    if (int st = adjoint_check(h, false)) return st;
    if (h->p.model != PFLBM_AC) return fail(h, PFLBM_EUNSUPPORTED, "the allocation-free adjoint covers the AC model");
    size_t need = 0;
    pflbm_adjoint_workspace_bytes(h, &need);
    if (need > (size_t)PFLBM_ADJOINT_SCRATCH_BYTES) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "the adjoint of this box needs %zu bytes of scratch, more than the "
                      "library's %zu (boxes of up to 128^3 nodes)", need, (size_t)PFLBM_ADJOINT_SCRATCH_BYTES);
        return fail(h, PFLBM_EINVAL, buf);
    }
    void* ptr = nullptr;
    HIPCHK(h, adjoint_scratch(h->device, &ptr), "adjoint scratch address");
    return adjoint_run(h, fwd_g, fwd_h, nullptr, lam_g, lam_h, nullptr, lam_g_out, lam_h_out, nullptr, dparams,
                       ptr);
}

// the workspace: phi [nodes], five adjoint values [5][nodes], block partials
// (laid out for float64; the float32 adjoint uses the same offsets)
extern "C++" template <class R>
static void adjoint_args(pflbm_t* h, void* work, AdjArgsT<R>& a) {
    const size_t nn = adj_nodes(h);
    std::memset(&a, 0, sizeof(a));
    const size_t blocks = (nn + 255) / 256;
    char* w = (char*)work;
    size_t off = 0;
    a.phi = (double*)(w + off);
    off += align_up(nn * 8, 256);
    a.work = (R*)(w + off);
    off += align_up(adj_nwork(h) * nn * 8, 256);
    a.partials = (double*)(w + off);
    off += align_up(blocks * 3 * 8, 256);
    if (h->p.model == PFLBM_NL) {
        a.nlpart = (double*)(w + off);
        off += align_up(blocks * 4 * 8, 256);
        a.nls = (double*)(w + off);
    }
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    for (int k = 0; k < 3; ++k) a.bc[k] = h->p.bc[k];
    a.qh = h->L.Qh;
    a.sigma = h->p.sigma;
    a.W = h->p.W;
    a.ph = h->ph;
}

static int adjoint_run(pflbm_t* h, const double* fwd_g, const double* fwd_h, const double* fwd_pu,
                       const double* lam_g, const double* lam_h, const double* lam_pu, double* lam_g_out,
                       double* lam_h_out, double* lam_pu_out, double* dparams, void* work) {
    if (!fwd_g || !fwd_h || !lam_g || !lam_h || !lam_g_out || !lam_h_out)
        return fail(h, PFLBM_EINVAL, "null pointer");
    if (lam_g_out == lam_g || lam_h_out == lam_h) return fail(h, PFLBM_EINVAL, "lambda in and out must not alias");
    AdjArgs a;
    adjoint_args(h, work, a);
    a.fg = fwd_g;
    a.fh = fwd_h;
    a.lg = lam_g;
    a.lh = lam_h;
    a.og = lam_g_out;
    a.oh = lam_h_out;
    a.fpu = fwd_pu;
    a.lpu = lam_pu;
    a.opu = lam_pu_out;
    HIPCHK(h, launch_adjoint(h->p.lattice, h->p.model, a, dparams, h->stream), "adjoint kernels");
    return PFLBM_OK;
}

// the float32 adjoint covers the AC model and, through the (phi u) forms,
// the CH model; with_pu selects the form asked for
static int adjoint_check_f32(pflbm_t* h, bool with_pu) {
    if (int st = guard(h)) return st;
    if (h->p.model != PFLBM_AC && h->p.model != PFLBM_CH)
        return fail(h, PFLBM_EUNSUPPORTED, "the float32 adjoint covers the AC and CH models");
    if (with_pu && h->p.model != PFLBM_CH)
        return fail(h, PFLBM_EUNSUPPORTED, "the AC model has no (phi u) state: use pflbm_adjoint_step_f32");
    return adjoint_check(h, with_pu);
}

static int adjoint_run_f32(pflbm_t* h, const float* fwd_g, const float* fwd_h, const float* fwd_pu,
                           const float* lam_g, const float* lam_h, const float* lam_pu, float* lam_g_out,
                           float* lam_h_out, float* lam_pu_out, double* dparams, void* work) {
    if (!fwd_g || !fwd_h || !lam_g || !lam_h || !lam_g_out || !lam_h_out || !work)
        return fail(h, PFLBM_EINVAL, "null pointer");
    if (lam_g_out == lam_g || lam_h_out == lam_h) return fail(h, PFLBM_EINVAL, "lambda in and out must not alias");
    AdjArgsT<float> a;
    adjoint_args(h, work, a);
    a.fg = fwd_g;
    a.fh = fwd_h;
    a.lg = lam_g;
    a.lh = lam_h;
    a.og = lam_g_out;
    a.oh = lam_h_out;
    a.fpu = fwd_pu;
    a.lpu = lam_pu;
    a.opu = lam_pu_out;
    HIPCHK(h, launch_adjoint_f32(h->p.lattice, h->p.model, a, dparams, h->stream), "adjoint kernels");
    return PFLBM_OK;
}

int pflbm_adjoint_step_f32(pflbm_t* h, const float* fwd_g, const float* fwd_h, const float* lam_g,
                           const float* lam_h, float* lam_g_out, float* lam_h_out, double* dparams, void* work) {
    if (int st = adjoint_check_f32(h, false)) return st;
    return adjoint_run_f32(h, fwd_g, fwd_h, nullptr, lam_g, lam_h, nullptr, lam_g_out, lam_h_out, nullptr, dparams,
                           work);
}

int pflbm_adjoint_step_pu_f32(pflbm_t* h, const float* fwd_g, const float* fwd_h, const float* fwd_pu,
                              const float* lam_g, const float* lam_h, const float* lam_pu, float* lam_g_out,
                              float* lam_h_out, float* lam_pu_out, double* dparams, void* work) {
    if (int st = adjoint_check_f32(h, true)) return st;
    if (!fwd_pu || !lam_pu || !lam_pu_out) return fail(h, PFLBM_EINVAL, "null pointer");
    if (lam_pu_out == lam_pu) return fail(h, PFLBM_EINVAL, "lambda in and out must not alias");
    return adjoint_run_f32(h, fwd_g, fwd_h, fwd_pu, lam_g, lam_h, lam_pu, lam_g_out, lam_h_out, lam_pu_out, dparams,
                           work);
}

int pflbm_adjoint_init_pu_f32(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                              const float* lam_g, const float* lam_h, const float* lam_pu, float* dphi0,
                              double* dparams, void* work) {
    if (int st = adjoint_check_f32(h, true)) return st;
    if (!phi0 || !lam_g || !lam_h || !lam_pu || !dphi0 || !work) return fail(h, PFLBM_EINVAL, "null pointer");
    AdjArgsT<float> a;
    adjoint_args(h, work, a);
    a.lg = lam_g;
    a.lh = lam_h;
    a.lpu = lam_pu;
    a.dphi0 = dphi0;
    HIPCHK(h, launch_adjoint_init_ch_f32(h->p.lattice, a, phi0, u0, p0, dparams, h->stream), "adjoint init kernels");
    return PFLBM_OK;
}

int pflbm_adjoint_seed_phi_f32(pflbm_t* h, const float* dphi, float* lam_g, float* lam_h) {
    if (int st = guard(h)) return st;
    if (int st = adjoint_check_f32(h, h->p.model == PFLBM_CH)) return st;
    if (!dphi || !lam_g || !lam_h) return fail(h, PFLBM_EINVAL, "null pointer");
    HIPCHK(h, launch_adjoint_seed_f32(dphi, lam_g, lam_h, (long long)adj_nodes(h), h->L.Qg, h->L.Qh, h->stream),
           "adjoint seed kernel");
    return PFLBM_OK;
}

int pflbm_adjoint_init_f32(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                           const float* lam_g, const float* lam_h, float* dphi0) {
    if (int st = adjoint_check_f32(h, false)) return st;
    if (!phi0 || !lam_g || !lam_h || !dphi0) return fail(h, PFLBM_EINVAL, "null pointer");
    AdjInitArgsT<float> a;
    std::memset(&a, 0, sizeof(a));
    a.lg = lam_g;
    a.lh = lam_h;
    a.phi0 = phi0;
    a.u0 = u0;
    a.p0 = p0;
    a.dphi0 = dphi0;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    a.ph = h->ph;
    HIPCHK(h, launch_adjoint_init_f32(h->p.lattice, a, h->stream), "adjoint init kernel");
    return PFLBM_OK;
}

int pflbm_adjoint_seed_phi(pflbm_t* h, const double* dphi, double* lam_g, double* lam_h) {
    if (int st = adjoint_check(h, true)) return st;
    if (h->p.model == PFLBM_NL)
        return fail(h, PFLBM_EUNSUPPORTED, "the nonlocal phase field is corrected: use pflbm_adjoint_seed");
    if (!dphi || !lam_g || !lam_h) return fail(h, PFLBM_EINVAL, "null pointer");
    HIPCHK(h, launch_adjoint_seed(dphi, lam_g, lam_h, (long long)adj_nodes(h), h->L.Qg, h->L.Qh, h->stream),
           "adjoint seed kernel");
    return PFLBM_OK;
}

int pflbm_adjoint_seed(pflbm_t* h, const double* fwd_h, const double* dphi, double* lam_g, double* lam_h,
                       double* dparams, void* work) {
    if (int st = adjoint_check(h, true)) return st;
    if (h->p.model != PFLBM_NL) return pflbm_adjoint_seed_phi(h, dphi, lam_g, lam_h);
    if (!fwd_h || !dphi || !lam_g || !lam_h || !work) return fail(h, PFLBM_EINVAL, "null pointer");
    AdjArgs a;
    adjoint_args(h, work, a);
    a.fh = fwd_h;
    HIPCHK(h, launch_adjoint_seed_nl(h->p.lattice, a, dphi, lam_g, lam_h, dparams, h->stream), "adjoint seed kernels");
    return PFLBM_OK;
}

int pflbm_adjoint_init(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                       const double* lam_g, const double* lam_h, double* dphi0) {
    if (int st = adjoint_check(h, false)) return st;
    if (!phi0 || !lam_g || !lam_h || !dphi0) return fail(h, PFLBM_EINVAL, "null pointer");
    AdjInitArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lg = lam_g;
    a.lh = lam_h;
    a.phi0 = phi0;
    a.u0 = u0;
    a.p0 = p0;
    a.dphi0 = dphi0;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    a.ph = h->ph;
    HIPCHK(h, launch_adjoint_init(h->p.lattice, h->p.model, a, h->stream), "adjoint init kernel");
    return PFLBM_OK;
}

int pflbm_adjoint_init_pu(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                          const double* lam_g, const double* lam_h, const double* lam_pu, double* dphi0,
                          double* dparams, void* work) {
    if (int st = adjoint_check(h, true)) return st;
    if (h->p.model == PFLBM_L18) {
        // Eq. liang_feq and h_eq of Eq. liang_geq do not depend on sigma, M, W
        if (!phi0 || !lam_g || !lam_h || !lam_pu || !dphi0) return fail(h, PFLBM_EINVAL, "null pointer");
        AdjInitArgs a;
        std::memset(&a, 0, sizeof(a));
        a.lg = lam_g;
        a.lh = lam_h;
        a.lpu = lam_pu;
        a.phi0 = phi0;
        a.u0 = u0;
        a.p0 = p0;
        a.dphi0 = dphi0;
        a.nx = h->p.nx;
        a.ny = h->p.ny;
        a.nz = h->p.nz;
        a.ph = h->ph;
        HIPCHK(h, launch_adjoint_init(h->p.lattice, h->p.model, a, h->stream), "adjoint init kernel");
        return PFLBM_OK;
    }
    if (h->p.model != PFLBM_CH && h->p.model != PFLBM_L14)
        return pflbm_adjoint_init(h, phi0, u0, p0, lam_g, lam_h, dphi0);
    if (!phi0 || !lam_g || !lam_h || !lam_pu || !dphi0 || !work) return fail(h, PFLBM_EINVAL, "null pointer");
    AdjArgs a;
    adjoint_args(h, work, a);
    a.lg = lam_g;
    a.lh = lam_h;
    a.lpu = lam_pu;
    a.dphi0 = dphi0;
    HIPCHK(h, launch_adjoint_init_ch(h->p.lattice, h->p.model, a, phi0, u0, p0, dparams, h->stream),
           "adjoint init kernels");
    return PFLBM_OK;
}

static int phiu_check(pflbm_t* h, const void* buf) {
    int st = guard(h);
    if (st) return st;
    if (!h->L.pu_bytes) return fail(h, PFLBM_EUNSUPPORTED, "this model keeps no (phi u) state");
    if (!buf) return fail(h, PFLBM_EINVAL, "null pointer");
    if (!h->initialised) return fail(h, PFLBM_EINVAL, "pflbm_init not called");
    return PFLBM_OK;
}

int pflbm_get_phiu(pflbm_t* h, double* pu) {
    if (int st = phiu_check(h, pu)) return st;
    HIPCHK(h, launch_phiu_io(h->p.precision, true, h->base + h->L.off_pu, pu, h->L.P, h->p.nx, h->p.ny, h->p.nz,
                             h->stream), "phiu get kernel");
    return PFLBM_OK;
}

int pflbm_set_phiu(pflbm_t* h, const double* pu) {
    if (int st = phiu_check(h, pu)) return st;
    HIPCHK(h, launch_phiu_io(h->p.precision, false, h->base + h->L.off_pu, (double*)pu, h->L.P, h->p.nx, h->p.ny,
                             h->p.nz, h->stream), "phiu set kernel");
    return PFLBM_OK;
}

}  // extern "C"
