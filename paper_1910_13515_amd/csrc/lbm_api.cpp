// C ABI of the D3Q39 13-moment DDF lattice Boltzmann library (declared in
// include/lbm.h).  Host side: parameter validation, derived constants, arena
// layout, obstacle link masks, and the launch sequences of the device kernels.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "d3q39.h"
#include "launch.h"
#include "slot.h"

using namespace lbm13;

namespace {

thread_local std::string g_last_error = "no error";

constexpr int64_t kAlign = 256;
constexpr int kMaxGrid = 2048;  // persistent grid cap (blocks); sizes the statistics partials

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int64_t storage_bytes(int storage) { return storage == kStoreF64 ? 8 : storage == kStoreF32 ? 4 : 2; }
int64_t lam_bytes(int storage) { return storage == kStoreF64 ? 8 : 4; }

struct Layout {
    int64_t buf[2], lam, links, fields, partial, totals, stats, stat_out, failed, table, single, single_status;
    int64_t total;
};

Layout make_layout(const lbm_params &p)
{
    const int64_t n = (int64_t)p.nx * p.ny * p.nz;
    Layout L{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const int64_t pop_bytes = 2LL * kQ * n * storage_bytes(p.storage);
    L.buf[0] = take(pop_bytes);
    L.buf[1] = take(pop_bytes);
    L.lam = take((int64_t)kM * n * lam_bytes(p.storage));
    L.links = p.solid ? take(n * 8) : -1;
    L.fields = take(5 * n * 8);
    L.partial = take((int64_t)moments_partial_blocks(n) * 5 * 8);
    L.totals = take(5 * 8);
    L.stats = take((int64_t)kMaxGrid * kWavesPerBlock * kStatWords * 8);
    L.stat_out = take(kStatWords * 8);
    L.failed = take(8);
    L.table = take((int64_t)slot_table_bytes(1));
    L.single = take((kQ + kM) * 8);
    L.single_status = take(8);
    L.total = off;
    return L;
}

bool face_ok(int f) { return f == LBM_FACE_PERIODIC || f == LBM_FACE_EQUILIBRIUM || f == LBM_FACE_NEUMANN; }

// Returns an empty string when the parameters are acceptable.
std::string validate(const lbm_params *p)
{
    if (!p) return "params is NULL";
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "grid dimensions must be >= 1";
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    if (p->storage < LBM_STORE_FP64 || p->storage > LBM_STORE_FP16_SHIFTED) return "unknown storage mode";
    // the gathers address one velocity's plane (FP64 and FP16: 16- and
    // 4-byte records of f_i and g_i) or, in FP32, a velocity pair's two
    // arrays from one base with 32-bit byte offsets: n < 2^28 in FP64, 2^29
    // in FP32, 2^30 in FP16 (the row stores switch to 64-bit lane addresses
    // above 2^28 cells)
    if (2 * n * storage_bytes(p->storage) >= ((int64_t)1 << 32)) return "grid too large for this storage mode";
    if (p->shift_ref < 0 || p->shift_ref > 1) return "shift_ref must be 0 or 1";
    const int dims[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a) {
        const int lo = p->faces[2 * a], hi = p->faces[2 * a + 1];
        if (!face_ok(lo) || !face_ok(hi)) return "unknown face kind";
        if ((lo == LBM_FACE_PERIODIC) != (hi == LBM_FACE_PERIODIC))
            return "both faces of an axis must be periodic, or neither";
        if (lo != LBM_FACE_PERIODIC && dims[a] < 7) return "a non-periodic axis needs at least 7 cells";
    }
    if (!(p->gamma > 1.0 && p->gamma <= 5.0 / 3.0 + 1e-12)) return "gamma must satisfy 1 < gamma <= 5/3";
    if (!(p->mach >= 0.0) || !std::isfinite(p->mach)) return "mach must be finite and >= 0";
    if (!(p->rho_ref >= 0.0) || !(p->T_ref >= 0.0)) return "rho_ref and T_ref must be >= 0";
    if (!std::isfinite(p->tau)) return "tau must be finite";
    if (p->tau > 0.0 && p->tau < 0.5) return "tau must be >= 1/2";
    if (p->tau <= 0.0 && !(p->reynolds > 0.0 && p->length_ref > 0.0 && p->mach > 0.0))
        return "tau <= 0 needs reynolds > 0, length_ref > 0 and mach > 0";
    if (p->newton_maxit < 0 || p->newton_maxit > 1000) return "newton_maxit out of range";
    if (!(p->newton_tol >= 0.0) || !std::isfinite(p->newton_tol)) return "newton_tol must be finite and >= 0";
    if (p->root_finder < 0 || p->root_finder > 1) return "root_finder must be 0 (Newton) or 1 (secant)";
    if (p->root_finder == 1 && p->storage != LBM_STORE_FP64) return "the secant root finder needs FP64 storage";
    if (p->mach > 0.0) {
        const double du = std::sqrt(p->u_dir[0] * p->u_dir[0] + p->u_dir[1] * p->u_dir[1] + p->u_dir[2] * p->u_dir[2]);
        if (!(du > 0.0) || !std::isfinite(du)) return "u_dir must be a nonzero finite vector when mach > 0";
    }
    if ((p->init_rho != nullptr) != (p->init_u != nullptr) || (p->init_rho != nullptr) != (p->init_T != nullptr))
        return "init_rho, init_u and init_T must be all given or all NULL";
    return "";
}

double pow2_near(double x)
{
    if (!(x > 0.0) || !std::isfinite(x)) return 1.0;
    return std::ldexp(1.0, (int)std::lround(std::log2(x)));
}

}  // namespace

struct lbm_ctx {
    lbm_params params{};
    Layout layout{};
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    int storage = 0;
    SlotDesc desc{};
    SlotTable *d_table = nullptr;
    int grid = 8;
    int64_t steps = 0;
    int64_t fluid_cells = 0;
    double tau = 0.0, shear_response = 0.0, u_ref[3] = {0, 0, 0};
    std::string err = "no error";
};

namespace {

int fail(lbm_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_last_error = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail(ctx, LBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

template <class T>
T *at(char *arena, int64_t off)
{
    return reinterpret_cast<T *>(arena + off);
}

// Equilibrium of one state on the device (FP64), copied to host.
int device_equilibrium(lbm_ctx *c, double rho, const double u[3], double T, double out[kQ + kM])
{
    double *d_out = at<double>(c->arena, c->layout.single);
    int *d_st = at<int>(c->arena, c->layout.single_status);
    HIP_TRY(c, launch_single_equilibrium(rho, u, T, 1e-14, 200, d_out, d_st, c->stream));
    int st = 0;
    HIP_TRY(c, hipMemcpyAsync(out, d_out, sizeof(double) * (kQ + kM), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&st, d_st, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (st == kFailed) return fail(c, LBM_E_NONREALIZABLE, "reference state has no 13-moment equilibrium");
    return LBM_OK;
}

// Shear response K(T) of the rest-state equilibrium w (per unit density):
// the linear response of the equilibrium to u_y at rest is w_i (a xi_y +
// b xi_y |xi|^2), with (a, b) solving the 2x2 block of J for the targets'
// derivatives (1, (D+2) T); K = sum_i that response times xi_x^2 xi_y.
double shear_response(const double *w, double T)
{
    double j11 = 0, j12 = 0, j22 = 0, k1 = 0, k2 = 0;
    for (int i = 0; i < kQ; ++i) {
        const double cx = vel(i, 0), cy = vel(i, 1), cz = vel(i, 2);
        const double q = cx * cx + cy * cy + cz * cz;
        j11 += w[i] * cy * cy;
        j12 += w[i] * cy * cy * q;
        j22 += w[i] * cy * cy * q * q;
        k1 += w[i] * cx * cx * cy * cy;
        k2 += w[i] * cx * cx * cy * cy * q;
    }
    const double r1 = 1.0, r2 = 5.0 * T;
    const double det = j11 * j22 - j12 * j12;
    const double a = (r1 * j22 - j12 * r2) / det;
    const double b = (j11 * r2 - j12 * r1) / det;
    return a * k1 + b * k2;
}

// Model constants of the secant root finder: the inverse of the Jacobian
// J_kl = sum_i w_i phi_ik phi_il of the rest equilibrium w (per unit
// density) in its cubic-symmetric blocks (h00, h0s, hss, hst over
// (1, xi_a^2); h11, h1q, hqq over (xi_a, xi_a |xi|^2); hp for xi_a xi_b).
// Returns false if J is singular or does not have that block structure.
bool secant_model(const double *w, double h[8])
{
    double J[kM][2 * kM];
    for (int k = 0; k < kM; ++k)
        for (int l = 0; l < 2 * kM; ++l) J[k][l] = (l - kM == k) ? 1.0 : 0.0;
    for (int i = 0; i < kQ; ++i) {
        const double x = vel(i, 0), y = vel(i, 1), z = vel(i, 2), q = x * x + y * y + z * z;
        const double phi[kM] = {1, x, y, z, x * x, y * y, z * z, x * y, x * z, y * z, x * q, y * q, z * q};
        for (int k = 0; k < kM; ++k)
            for (int l = 0; l < kM; ++l) J[k][l] += w[i] * phi[k] * phi[l];
    }
    // Gauss-Jordan with partial pivoting on [J | I]
    for (int col = 0; col < kM; ++col) {
        int piv = col;
        for (int r = col + 1; r < kM; ++r)
            if (std::fabs(J[r][col]) > std::fabs(J[piv][col])) piv = r;
        if (!(std::fabs(J[piv][col]) > 0.0)) return false;
        for (int l = 0; l < 2 * kM; ++l) std::swap(J[col][l], J[piv][l]);
        const double inv = 1.0 / J[col][col];
        for (int l = 0; l < 2 * kM; ++l) J[col][l] *= inv;
        for (int r = 0; r < kM; ++r)
            if (r != col) {
                const double f = J[r][col];
                for (int l = 0; l < 2 * kM; ++l) J[r][l] -= f * J[col][l];
            }
    }
    auto H = [&](int k, int l) { return J[k][kM + l]; };
    h[0] = H(0, 0);
    h[1] = H(0, 4);
    h[2] = H(4, 4);
    h[3] = H(4, 5);
    h[4] = H(1, 1);
    h[5] = H(1, 10);
    h[6] = H(10, 10);
    h[7] = H(7, 7);
    // the structure the kernel assumes (cubic symmetry of the lattice and of
    // the rest weights; odd and even functions decouple)
    double big = 0.0, dev = 0.0;
    for (int k = 0; k < kM; ++k)
        for (int l = 0; l < kM; ++l) {
            const auto deg = [](int m) { return m == 0 ? 0 : m <= 3 ? 1 : m <= 9 ? 2 : 3; };
            const auto axis = [](int m) { return m >= 1 && m <= 3 ? m - 1 : m >= 10 ? m - 10 : m >= 4 && m <= 6 ? m - 4 : -1; };
            double ref = 0.0;
            const bool ek = deg(k) % 2 == 0, el = deg(l) % 2 == 0;
            if (ek && el) {
                const bool dk = k == 0 || (k >= 4 && k <= 6), dl = l == 0 || (l >= 4 && l <= 6);
                if (dk && dl) {
                    if (k == 0 && l == 0) ref = h[0];
                    else if (k == 0 || l == 0) ref = h[1];
                    else ref = k == l ? h[2] : h[3];
                } else if (k == l) {
                    ref = h[7];
                }
            } else if (!ek && !el && axis(k) == axis(l)) {
                ref = (k == l) ? (k <= 3 ? h[4] : h[6]) : h[5];
            }
            big = std::max(big, std::fabs(H(k, l)));
            dev = std::max(dev, std::fabs(H(k, l) - ref));
        }
    return std::isfinite(big) && dev <= 1e-10 * big;
}

// Per-cell link mask for half-way bounce-back: bit i set when a lattice node
// passed over by velocity i (x - k dir_i, k = 1..mult_i) is solid; bit 63 for
// solid cells.  Computed for fluid cells only.
void build_links(const lbm_params &p, std::vector<uint64_t> &links)
{
    const int64_t nx = p.nx, ny = p.ny, nz = p.nz, n = nx * ny * nz;
    links.assign(n, 0);
    const int dims[3] = {p.nx, p.ny, p.nz};
    bool periodic[3];
    for (int a = 0; a < 3; ++a) periodic[a] = p.faces[2 * a] == LBM_FACE_PERIODIC;
    auto wrap = [&](int v, int a) {
        if (!periodic[a]) return v;
        const int m = dims[a];
        v %= m;
        return v < 0 ? v + m : v;
    };
    auto fluid_coord = [&](int x, int y, int z) {
        const int c[3] = {x, y, z};
        for (int a = 0; a < 3; ++a)
            if (!periodic[a] && (c[a] < 3 || c[a] >= dims[a] - 3)) return false;
        return true;
    };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t cell = x + nx * (y + ny * (int64_t)z);
                if (p.solid[cell]) {
                    links[cell] = 1ull << 63;
                    continue;
                }
                if (!fluid_coord(x, y, z)) continue;
                uint64_t m = 0;
                for (int i = 1; i < kQ; ++i) {
                    const int c[3] = {vel(i, 0), vel(i, 1), vel(i, 2)};
                    const int mult = std::max({std::abs(c[0]), std::abs(c[1]), std::abs(c[2])});
                    for (int k = 1; k <= mult; ++k) {
                        const int sx = wrap(x - k * (c[0] / mult), 0);
                        const int sy = wrap(y - k * (c[1] / mult), 1);
                        const int sz = wrap(z - k * (c[2] / mult), 2);
                        if (p.solid[sx + nx * (sy + ny * (int64_t)sz)]) {
                            m |= 1ull << i;
                            break;
                        }
                    }
                }
                links[cell] = m;
            }
}

// Everything lbm_create does once the context exists: defaults, derived
// constants, obstacle links, the initial equilibrium, the slot table and the
// persistent grid.  On failure c->err holds the message; the caller frees c.
int create_in(lbm_ctx *c, const lbm_params *params)
{
    const Layout &L = c->layout;
    lbm_params &p = c->params;
    if (p.rho_ref == 0.0) p.rho_ref = 1.0;
    if (p.T_ref == 0.0) p.T_ref = 0.5;
    // the secant variant takes more (cheaper) updates than Newton
    if (p.newton_maxit == 0) p.newton_maxit = p.root_finder == 1 ? 100 : 20;
    // FP32 arithmetic: 1e-5 of the largest target.  From the warm start one
    // Newton update reaches it in all but a few cells; tighter bounds (down
    // to the FP32 residual floor near 1e-6) add a second update to most waves
    // without lowering the error against FP64, which storage rounding sets.
    if (p.newton_tol == 0.0) p.newton_tol = p.storage == LBM_STORE_FP64 ? 1e-12 : 1e-5;

    const double Cv = 1.0 / (p.gamma - 1.0);
    const double delta = 2.0 * Cv - 3.0;
    const double cs = std::sqrt(p.gamma * p.T_ref);
    if (p.mach > 0.0) {
        const double du = std::sqrt(p.u_dir[0] * p.u_dir[0] + p.u_dir[1] * p.u_dir[1] + p.u_dir[2] * p.u_dir[2]);
        for (int a = 0; a < 3; ++a) c->u_ref[a] = p.mach * cs * p.u_dir[a] / du;
    }

    // rest-state equilibrium at T_ref (shear response, rest shift weights)
    double rest[kQ + kM], stream_eq[kQ + kM];
    const double zero[3] = {0.0, 0.0, 0.0};
    int rc = device_equilibrium(c, 1.0, zero, p.T_ref, rest);
    if (rc != LBM_OK) return rc;
    rc = device_equilibrium(c, p.rho_ref, c->u_ref, p.T_ref, stream_eq);
    if (rc != LBM_OK) return rc;
    c->shear_response = shear_response(rest, p.T_ref);

    if (p.tau > 0.0) {
        c->tau = p.tau;
    } else {
        const double speed = p.mach * cs;
        c->tau = 0.5 + speed * p.length_ref / (p.reynolds * c->shear_response);
    }

    SlotDesc &d = c->desc;
    std::memset(&d, 0, sizeof(d));
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.nsegx = (p.nx + kSegment - 1) / kSegment;
    d.n = (int64_t)p.nx * p.ny * p.nz;
    d.segments = (int64_t)d.nsegx * p.ny * p.nz;
    d.blocks = (int32_t)((d.segments + kWavesPerBlock - 1) / kWavesPerBlock);
    for (int a = 0; a < 3; ++a) {
        const int lo = p.faces[2 * a], hi = p.faces[2 * a + 1];
        d.axis[a] = lo == LBM_FACE_PERIODIC ? kAxisPeriodic : kAxisOpen;
        d.open_lo[a] = lo != LBM_FACE_PERIODIC;
        d.open_hi[a] = hi != LBM_FACE_PERIODIC;
        d.neumann_lo[a] = lo == LBM_FACE_NEUMANN;
        d.neumann_hi[a] = hi == LBM_FACE_NEUMANN;
    }
    d.has_links = params->solid != nullptr;
    d.kn_relax = p.kn_relax ? 1 : 0;
    d.root_finder = p.root_finder;
    d.qn_T_ref = p.T_ref;
    if (p.root_finder == 1 && !secant_model(rest, d.qn_h))
        return fail(c, LBM_E_NONREALIZABLE, "the rest Jacobian at T_ref is not usable for the secant root finder");
    d.maxit = p.newton_maxit;
    d.maxit_cold = std::max(p.newton_maxit, 100);
    d.parity0 = 0;
    d.steps_todo = 0x7fffffff;
    d.storage = p.storage;
    d.tol = p.newton_tol;
    {
        const double t1 = c->tau * 1.05, t2 = c->tau * 1.35;
        d.omega[0] = 1.0 / c->tau;
        d.omega[1] = 1.0 / t1;
        d.omega[2] = 1.0 / t2;
        d.omega[3] = 1.0;  // alpha = 1/tau: the cell is replaced by its equilibrium
    }
    d.delta = delta;
    d.two_cv = 2.0 * Cv;
    d.buf[0] = c->arena + L.buf[0];
    d.buf[1] = c->arena + L.buf[1];
    d.lam = c->arena + L.lam;
    d.links = params->solid ? at<uint64_t>(c->arena, L.links) : nullptr;
    d.stats = at<int64_t>(c->arena, L.stats);
    if (p.storage != LBM_STORE_FP64) {
        double w[2 * kQ];
        for (int i = 0; i < kQ; ++i) {
            w[i] = p.shift_ref ? stream_eq[i] : p.rho_ref * rest[i];
            w[kQ + i] = delta * p.T_ref * w[i];
        }
        double mass = 0, mom[3] = {0, 0, 0}, ener = 0;
        // shift weights on a 2^-21 grid: every weight and every sum of the
        // weights below (all < 8 in magnitude) is then exact in FP32, so the
        // FP32 moments carry no constant rounding bias from the shift
        for (int i = 0; i < 2 * kQ; ++i) d.shift_w[i] = (float)(std::nearbyint(std::ldexp(w[i], 21)) * std::ldexp(1.0, -21));
        // FP16: one power-of-two scale per velocity shell, from the rest-state
        // weight of the shell (g: times delta T_ref when delta > 0); FP32: 1
        for (int sh = 0; sh < 6; ++sh) {
            double sf = 1.0, sg = 1.0;
            if (p.storage == LBM_STORE_FP16_SHIFTED) {
                for (int i = 0; i < kQ; ++i)
                    if (shell(i) == sh) sf = pow2_near(p.rho_ref * rest[i]);
                sg = delta > 0.0 ? sf * pow2_near(delta * p.T_ref) : sf;
            }
            d.shell_scale[0][sh] = (float)sf;
            d.shell_scale[1][sh] = (float)sg;
            d.shell_inv_scale[0][sh] = (float)(1.0 / sf);
            d.shell_inv_scale[1][sh] = (float)(1.0 / sg);
        }
        for (int i = 0; i < kQ; ++i) {
            const double wf = (double)d.shift_w[i], wg = (double)d.shift_w[kQ + i];
            const int cx = vel(i, 0), cy = vel(i, 1), cz = vel(i, 2);
            mass += wf;
            mom[0] += wf * cx;
            mom[1] += wf * cy;
            mom[2] += wf * cz;
            ener += wf * (cx * cx + cy * cy + cz * cz) + wg;
        }
        // bounce-back correction for unequal weights of opposite velocities
        // (the weights lie on a 2^-21 grid, so the differences are exact)
        d.asym_bounce = 0;
        for (int i = 0; i < 2 * kQ; ++i) {
            const int v = i % kQ, o = (i < kQ ? 0 : kQ) + opposite(v);
            d.bb_corr[i] = d.shift_w[o] - d.shift_w[i];
            if (d.bb_corr[i] != 0.0f && d.has_links) d.asym_bounce = 1;
        }
        d.ref_mass = (float)mass;
        d.ref_mom[0] = (float)mom[0];
        d.ref_mom[1] = (float)mom[1];
        d.ref_mom[2] = (float)mom[2];
        d.ref_energy = (float)ener;
    }

    // obstacle links
    const int64_t n = d.n;
    if (params->solid) {
        std::vector<uint64_t> links;
        build_links(*params, links);
        HIP_TRY(c, hipMemcpyAsync(at<uint64_t>(c->arena, L.links), links.data(), n * 8, hipMemcpyHostToDevice,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    {
        int64_t fluid = 0;
        for (int64_t z = 0; z < p.nz; ++z)
            for (int64_t y = 0; y < p.ny; ++y)
                for (int64_t x = 0; x < p.nx; ++x) {
                    const int64_t cc[3] = {x, y, z};
                    const int64_t dims[3] = {p.nx, p.ny, p.nz};
                    bool f = !(params->solid && params->solid[x + p.nx * (y + p.ny * z)]);
                    for (int a = 0; a < 3 && f; ++a)
                        if (d.open_lo[a] && (cc[a] < 3 || cc[a] >= dims[a] - 3)) f = false;
                    fluid += f;
                }
        c->fluid_cells = fluid;
    }

    // initial fields -> equilibrium state
    {
        std::vector<double> host(5 * n);
        for (int64_t i = 0; i < n; ++i) {
            host[i] = params->init_rho ? params->init_rho[i] : p.rho_ref;
            host[n + i] = params->init_u ? params->init_u[i] : c->u_ref[0];
            host[2 * n + i] = params->init_u ? params->init_u[n + i] : c->u_ref[1];
            host[3 * n + i] = params->init_u ? params->init_u[2 * n + i] : c->u_ref[2];
            host[4 * n + i] = params->init_T ? params->init_T[i] : p.T_ref;
        }
        for (int64_t i = 0; i < n; ++i)
            if (!(host[i] > 0.0) || !(host[4 * n + i] > 0.0) || !std::isfinite(host[i] + host[n + i] + host[2 * n + i] +
                                                                                 host[3 * n + i] + host[4 * n + i])) {
                c->err = "initial fields need finite values with rho > 0 and T > 0";
                return LBM_E_INVAL;
            }
        double *d_fields = at<double>(c->arena, L.fields);
        unsigned long long *d_failed = at<unsigned long long>(c->arena, L.failed);
        HIP_TRY(c, hipMemcpyAsync(d_fields, host.data(), 5 * n * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemsetAsync(d_failed, 0, 8, c->stream));
        SlotDesc di = d;
        // the initial equilibrium is always solved in FP64 to the FP64 bound
        di.tol = p.storage == LBM_STORE_FP64 ? p.newton_tol : 1e-12;
        HIP_TRY(c, launch_init(p.storage, di, d_fields, d_failed, c->stream));
        unsigned long long failed = 0;
        HIP_TRY(c, hipMemcpyAsync(&failed, d_failed, 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (failed) {
            c->err = std::to_string(failed) + " initial cells have no 13-moment equilibrium";
            return LBM_E_NONREALIZABLE;
        }
    }

    // slot table (one slot) and persistent grid
    {
        std::vector<char> tab(slot_table_bytes(1), 0);
        SlotTable *t = reinterpret_cast<SlotTable *>(tab.data());
        t->nslots = 1;
        t->total_blocks = d.blocks;
        t->block_start[0] = 0;
        t->block_start[1] = d.blocks;
        t->slot[0] = d;
        c->d_table = at<SlotTable>(c->arena, L.table);
        HIP_TRY(c, hipMemcpyAsync(c->d_table, tab.data(), tab.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        int dev = 0, per_cu = 1;
        hipDeviceProp_t prop;
        HIP_TRY(c, hipGetDevice(&dev));
        HIP_TRY(c, hipGetDeviceProperties(&prop, dev));
        HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step_kernel_symbol(p.storage),
                                                                 kBlockThreads, 0));
        int grid = std::max(1, per_cu) * prop.multiProcessorCount;
        const int need = (d.blocks + 7) / 8 * 8;
        grid = std::min(grid, need);
        grid = std::min(grid, kMaxGrid);
        grid = std::max(8, grid / 8 * 8);
        c->grid = grid;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_version(void) { return 10100; }

int lbm_velocities(int32_t *out)
{
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    for (int i = 0; i < kQ; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = vel(i, a);
    return LBM_OK;
}

int64_t lbm_required_bytes(const lbm_params *params)
{
    const std::string v = validate(params);
    if (!v.empty()) return fail(nullptr, LBM_E_INVAL, v);
    return make_layout(*params).total;
}

int lbm_create(const lbm_params *params, void *dev_arena, int64_t arena_bytes, void *hip_stream, lbm_ctx **out)
{
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    const std::string v = validate(params);
    if (!v.empty()) return fail(nullptr, LBM_E_INVAL, v);
    if (!dev_arena) return fail(nullptr, LBM_E_INVAL, "dev_arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign != 0)
        return fail(nullptr, LBM_E_INVAL, "dev_arena must be 256-byte aligned");
    const Layout L = make_layout(*params);
    if (arena_bytes < L.total)
        return fail(nullptr, LBM_E_NOMEM,
                    "arena of " + std::to_string(arena_bytes) + " bytes < required " + std::to_string(L.total));

    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return fail(nullptr, LBM_E_DEVICE, "no HIP device");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(nullptr, LBM_E_DEVICE, std::string("library built for gfx950, device is ") + prop.gcnArchName);
    }

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    c->params = *params;
    c->params.solid = nullptr;
    c->params.init_rho = c->params.init_u = c->params.init_T = nullptr;
    c->layout = L;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->arena = static_cast<char *>(dev_arena);
    c->storage = params->storage;
    const int rc = create_in(c, params);
    if (rc != LBM_OK) {
        g_last_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int32_t nsteps, lbm_step_stats *stats)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps must be >= 0");
    int64_t *d_stats = at<int64_t>(c->arena, c->layout.stats);
    const int nwaves = c->grid * kWavesPerBlock;
    if (stats) HIP_TRY(c, launch_zero(d_stats, (int64_t)nwaves * kStatWords, c->stream));
    for (int32_t s = 0; s < nsteps; ++s) {
        const int j = (int)((c->steps + s) & 1);
        // statistics only when asked for: the kernels without them run lighter
        HIP_TRY(c, launch_step(c->storage, c->d_table, c->grid, j, stats ? d_stats : nullptr, c->stream,
                               c->params.root_finder, c->desc.n >= kWideCells));
    }
    c->steps += nsteps;
    if (!stats) return LBM_OK;
    int64_t *d_out = at<int64_t>(c->arena, c->layout.stat_out);
    HIP_TRY(c, launch_reduce_stats(d_stats, nwaves, d_out, c->stream));
    int64_t h[kStatWords];
    HIP_TRY(c, hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    stats->cell_updates = c->fluid_cells * (int64_t)nsteps;
    stats->iterations = h[0];
    stats->max_iterations = h[1];
    stats->failed = h[2];
    stats->cold_restarts = h[3];
    for (int k = 0; k < 4; ++k) stats->alpha_hist[k] = h[4 + k];
    stats->wave_iterations = h[8];
    // every lane of a wave adds the wave's count once per wave-step
    stats->waves = h[9];
    if (h[2] > 0) return fail(c, LBM_E_NEWTON, std::to_string(h[2]) + " cell updates did not converge");
    return LBM_OK;
}

int lbm_moments(lbm_ctx *c, double *out_host, double *totals)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    const int64_t n = c->desc.n;
    double *d_fields = at<double>(c->arena, c->layout.fields);
    double *d_partial = at<double>(c->arena, c->layout.partial);
    double *d_totals = at<double>(c->arena, c->layout.totals);
    HIP_TRY(c, launch_moments(c->storage, c->desc, (int)(c->steps & 1), d_fields, d_partial, d_totals, c->stream));
    double t[5];
    if (out_host) HIP_TRY(c, hipMemcpyAsync(out_host, d_fields, 5 * n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(t, d_totals, sizeof(t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (totals)
        for (int k = 0; k < 5; ++k) totals[k] = t[k];
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(t[k])) return fail(c, LBM_E_NONFINITE, "non-finite moments in fluid cells");
    return LBM_OK;
}

int lbm_moments_noalloc(lbm_ctx *c, double *dev_out, double *totals)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!dev_out) return fail(c, LBM_E_INVAL, "dev_out is NULL (5*N doubles of device memory are required)");
    const int64_t n = c->desc.n;
    if (n > kNoallocMaxCells)
        return fail(c, LBM_E_INVAL, "lbm_moments_noalloc takes grids of at most " + std::to_string(kNoallocMaxCells) +
                                        " cells; this one has " + std::to_string(n) + " (use lbm_moments)");
    double *scr = nullptr;
    HIP_TRY(c, noalloc_scratch(&scr));
    const int64_t nb = (kNoallocMaxCells + 255) / 256;
    HIP_TRY(c, launch_moments(c->storage, c->desc, (int)(c->steps & 1), dev_out, scr, scr + nb * 5, c->stream));
    double t[5];
    HIP_TRY(c, hipMemcpyAsync(t, scr + nb * 5, sizeof(t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (totals)
        for (int k = 0; k < 5; ++k) totals[k] = t[k];
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(t[k])) return fail(c, LBM_E_NONFINITE, "non-finite moments in fluid cells");
    return LBM_OK;
}

int lbm_diagnostics(lbm_ctx *c, double *eps_out, int32_t *iters_out)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    const int64_t n = c->desc.n;
    double *d_diag = at<double>(c->arena, c->layout.fields);  // 2n of the 5n moment doubles
    const int grid = (int)std::min<int64_t>(c->desc.blocks, kMaxGrid);
    HIP_TRY(c, launch_diag(c->storage, c->d_table, std::max(grid, 1), (int)(c->steps & 1), d_diag, c->stream));
    if (eps_out) HIP_TRY(c, hipMemcpyAsync(eps_out, d_diag, n * 8, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> it;
    if (iters_out) {
        it.resize(n);
        HIP_TRY(c, hipMemcpyAsync(it.data(), d_diag + n, n * 8, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (iters_out)
        for (int64_t k = 0; k < n; ++k) iters_out[k] = (int32_t)it[k];
    return LBM_OK;
}

int lbm_get_state(lbm_ctx *c, double *f, double *g, double *lam)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    const int64_t n = c->desc.n;
    double *d_fields = at<double>(c->arena, c->layout.fields);
    const int parity = (int)(c->steps & 1);
    for (int pop = 0; pop < 2 * kQ; ++pop) {
        double *dst = pop < kQ ? f : g;
        if (!dst) continue;
        HIP_TRY(c, launch_decode_pop(c->storage, c->desc, parity, pop, d_fields, c->stream));
        HIP_TRY(c, hipMemcpyAsync(dst + (int64_t)(pop % kQ) * n, d_fields, n * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (lam) {
        for (int k = 0; k < kM; ++k) {
            HIP_TRY(c, launch_copy_lam(c->storage, c->desc, k, 0, d_fields, c->stream));
            HIP_TRY(c, hipMemcpyAsync(lam + (int64_t)k * n, d_fields, n * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
    }
    return LBM_OK;
}

int lbm_set_state(lbm_ctx *c, const double *f, const double *g, const double *lam)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!f || !g || !lam) return fail(c, LBM_E_INVAL, "f, g and lam are required");
    const int64_t n = c->desc.n;
    double *d_fields = at<double>(c->arena, c->layout.fields);
    for (int pop = 0; pop < 2 * kQ; ++pop) {
        const double *srcp = (pop < kQ ? f : g) + (int64_t)(pop % kQ) * n;
        HIP_TRY(c, hipMemcpyAsync(d_fields, srcp, n * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, launch_encode_pop(c->storage, c->desc, pop, d_fields, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    for (int k = 0; k < kM; ++k) {
        HIP_TRY(c, hipMemcpyAsync(d_fields, lam + (int64_t)k * n, n * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, launch_copy_lam(c->storage, c->desc, k, 1, d_fields, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    c->steps = 0;
    return LBM_OK;
}

int lbm_get_info(const lbm_ctx *c, lbm_info *info)
{
    if (!c || !info) return fail(nullptr, LBM_E_INVAL, "ctx or info is NULL");
    info->tau = c->tau;
    for (int a = 0; a < 3; ++a) info->u_ref[a] = c->u_ref[a];
    info->shear_response = c->shear_response;
    info->delta = c->desc.delta;
    info->cells = c->desc.n;
    info->fluid_cells = c->fluid_cells;
    info->steps_done = c->steps;
    info->arena_bytes_used = c->layout.total;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *c)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    const hipError_t e = hipStreamSynchronize(c->stream);
    delete c;
    if (e != hipSuccess) return fail(nullptr, LBM_E_DEVICE, hipGetErrorString(e));
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving pool
// ---------------------------------------------------------------------------
namespace {

struct PoolSlot {
    bool used = false;
    bool in_round = false;  // part of the launched, not yet waited-for round
    lbm_ctx *ctx = nullptr;
    int64_t off = 0, bytes = 0;
    int64_t steps_total = 0, steps_left = 0;
    int64_t admitted_seq = 0;  // admission order (ties of the orders below)
    double admitted_at = 0.0;  // host clock at admission (s)
};

// first-fit allocator over [base, base + size) in 256-byte units
struct RangeHeap {
    std::map<int64_t, int64_t> free_;  // offset -> size
    void init(int64_t base, int64_t size)
    {
        free_.clear();
        if (size > 0) free_[base] = size;
    }
    int64_t alloc(int64_t bytes)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0) free_[off + bytes] = rest;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t total() const
    {
        int64_t t = 0;
        for (auto &kv : free_) t += kv.second;
        return t;
    }
    int64_t largest() const
    {
        int64_t t = 0;
        for (auto &kv : free_) t = std::max(t, kv.second);
        return t;
    }
};

}  // namespace

struct lbm_pool {
    int storage = 0, max_slots = 0, graph_steps = 1, grid = 8, sched = LBM_SCHED_ALL;
    int64_t fill_cells = 0;
    double rate = 4e9;          // cell updates per second of recent rounds (LBM_SCHED_VFT)
    double launched_at = 0.0;   // host clock of the round in flight
    hipStream_t stream = nullptr;        // rounds (the captured graph)
    hipStream_t admit_stream = nullptr;  // admission, moments, release
    hipEvent_t admitted = nullptr;       // last admission's work, waited for by the next round
    bool own_stream = false;
    bool in_flight = false;
    char *arena = nullptr;
    int64_t arena_bytes = 0;
    SlotTable *d_table = nullptr;
    SlotTable *h_table = nullptr;  // pinned host copy
    size_t table_bytes = 0;
    RangeHeap heap;
    std::vector<PoolSlot> slots;
    std::vector<int> round;  // slots of the launched round
    int64_t seq = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    mutable std::string err = "no error";  // also set by the const queries
};

namespace {

int pool_fail(lbm_pool *p, int code, const std::string &msg)
{
    if (p) p->err = msg;
    else g_last_error = msg;
    return code;
}

#define POOL_TRY(pool, expr)                                                                            \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return pool_fail(pool, LBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

void pool_free(lbm_pool *p)
{
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->admit_stream) (void)hipStreamSynchronize(p->admit_stream);
    for (auto &s : p->slots)
        if (s.used && s.ctx) lbm_destroy(s.ctx);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->h_table) (void)hipHostFree(p->h_table);
    if (p->admitted) (void)hipEventDestroy(p->admitted);
    if (p->admit_stream) (void)hipStreamDestroy(p->admit_stream);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

bool slot_ok(const lbm_pool *p, int32_t slot) { return p && slot >= 0 && slot < p->max_slots && p->slots[slot].used; }

// Error of a slot-level call: the pool's message when there is a pool.
int slot_fail(const lbm_pool *p)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "pool is NULL");
    p->err = "invalid slot";
    return LBM_E_INVAL;
}

double host_seconds()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The slots the next round advances.  LBM_SCHED_ALL: every slot with steps
// left (processor sharing).  LBM_SCHED_SRPT: slots in order of remaining work
// (fluid cells x steps left).  LBM_SCHED_VFT: slots in order of virtual finish
// time, admission time + remaining work / recent throughput (small solves
// still go first, but a large one is not passed by solves admitted after it
// would have finished alone).  Ties by admission order.  For both orders the
// first slot always runs and the next ones join while the cells per step stay
// within the first slot's plus fill_cells: a launch is never slowed down by
// more than what fills the device anyway.
std::vector<int> pick_round(const lbm_pool *p)
{
    std::vector<int> run;
    for (int i = 0; i < p->max_slots; ++i)
        if (p->slots[i].used && p->slots[i].steps_left > 0) run.push_back(i);
    if (p->sched == LBM_SCHED_ALL || run.size() < 2) return run;
    auto work = [&](int i) { return (double)p->slots[i].ctx->fluid_cells * (double)p->slots[i].steps_left; };
    auto key = [&](int i) {
        return p->sched == LBM_SCHED_SRPT ? work(i) : p->slots[i].admitted_at + work(i) / p->rate;
    };
    std::sort(run.begin(), run.end(), [&](int a, int b) {
        const double ka = key(a), kb = key(b);
        return ka != kb ? ka < kb : p->slots[a].admitted_seq < p->slots[b].admitted_seq;
    });
    const int64_t cap = p->slots[run[0]].ctx->desc.n + p->fill_cells;
    std::vector<int> out;
    int64_t cells = 0;
    for (int i : run) {
        const int64_t c = p->slots[i].ctx->desc.n;
        if (!out.empty() && cells + c > cap) continue;
        out.push_back(i);
        cells += c;
    }
    return out;
}

}  // namespace

extern "C" {

int64_t lbm_pool_overhead_bytes(int32_t max_slots)
{
    if (max_slots < 1 || max_slots > kMaxSlots) return fail(nullptr, LBM_E_INVAL, "max_slots out of range");
    return align_up((int64_t)slot_table_bytes(max_slots));
}

int lbm_pool_create(int32_t storage, int32_t max_slots, int32_t graph_steps, int32_t sched, int64_t fill_cells,
                    void *dev_arena, int64_t arena_bytes, void *hip_stream, lbm_pool **out)
{
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (storage < LBM_STORE_FP64 || storage > LBM_STORE_FP16_SHIFTED) return fail(nullptr, LBM_E_INVAL, "unknown storage");
    if (max_slots < 1 || max_slots > kMaxSlots) return fail(nullptr, LBM_E_INVAL, "max_slots out of range");
    if (graph_steps < 1 || graph_steps > 4096) return fail(nullptr, LBM_E_INVAL, "graph_steps out of range");
    if (sched != LBM_SCHED_ALL && sched != LBM_SCHED_SRPT && sched != LBM_SCHED_VFT)
        return fail(nullptr, LBM_E_INVAL, "unknown scheduling policy");
    if (fill_cells < 0) return fail(nullptr, LBM_E_INVAL, "fill_cells must be >= 0");
    if (!dev_arena || reinterpret_cast<uintptr_t>(dev_arena) % kAlign != 0)
        return fail(nullptr, LBM_E_INVAL, "dev_arena must be a 256-byte aligned device pointer");
    const int64_t head = lbm_pool_overhead_bytes(max_slots);
    if (arena_bytes < head) return fail(nullptr, LBM_E_NOMEM, "arena smaller than the pool overhead");

    lbm_pool *p = new (std::nothrow) lbm_pool();
    if (!p) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    p->storage = storage;
    p->max_slots = max_slots;
    p->graph_steps = graph_steps;
    p->sched = sched;
    p->arena = static_cast<char *>(dev_arena);
    p->arena_bytes = arena_bytes;
    p->table_bytes = slot_table_bytes(max_slots);
    p->d_table = reinterpret_cast<SlotTable *>(p->arena);
    p->heap.init(head, arena_bytes - head);
    p->slots.resize(max_slots);
    auto bail = [&](int code, const std::string &msg) {
        g_last_error = msg;
        pool_free(p);
        return code;
    };
    if (hip_stream) {
        p->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        const hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(LBM_E_DEVICE, std::string("pool stream: ") + hipGetErrorString(e));
        p->own_stream = true;
    }
    {
        hipError_t e = hipStreamCreateWithFlags(&p->admit_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(LBM_E_DEVICE, std::string("admission stream: ") + hipGetErrorString(e));
        e = hipEventCreateWithFlags(&p->admitted, hipEventDisableTiming);
        if (e != hipSuccess) return bail(LBM_E_DEVICE, std::string("admission event: ") + hipGetErrorString(e));
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&p->h_table), p->table_bytes, hipHostMallocDefault) != hipSuccess)
        return bail(LBM_E_DEVICE, "hipHostMalloc failed");
    std::memset(p->h_table, 0, p->table_bytes);
    if (hipMemcpyAsync(p->d_table, p->h_table, p->table_bytes, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return bail(LBM_E_DEVICE, "slot table upload failed");
    {
        int dev = 0, per_cu = 1;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return bail(LBM_E_DEVICE, "no HIP device");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return bail(LBM_E_DEVICE, std::string("library built for gfx950, device is ") + prop.gcnArchName);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step_kernel_symbol(storage), kBlockThreads, 0) !=
            hipSuccess)
            return bail(LBM_E_DEVICE, "occupancy query failed");
        int grid = std::max(1, per_cu) * prop.multiProcessorCount;
        grid = std::min(grid, kMaxGrid);
        p->grid = std::max(8, grid / 8 * 8);
    }
    // default fill: four row blocks per resident workgroup of the persistent grid
    p->fill_cells = fill_cells > 0 ? fill_cells : (int64_t)p->grid * kBlockThreads * 4;
    // capture graph_steps launches of the batched step; the slot table (read
    // by the kernel at run time) decides which slots each launch advances
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(LBM_E_DEVICE, "hipStreamBeginCapture failed");
    for (int j = 0; j < graph_steps; ++j) {
        if (launch_step(storage, p->d_table, p->grid, j, nullptr, p->stream) != hipSuccess) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(p->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return bail(LBM_E_DEVICE, "kernel launch during capture failed");
        }
    }
    if (hipStreamEndCapture(p->stream, &p->graph) != hipSuccess) return bail(LBM_E_DEVICE, "hipStreamEndCapture failed");
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(LBM_E_DEVICE, "hipGraphInstantiate failed");
    *out = p;
    return LBM_OK;
}

int lbm_pool_admit(lbm_pool *p, const lbm_params *params, int32_t nsteps, int32_t *slot_out)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "pool is NULL");
    if (!params || !slot_out || nsteps < 0) return pool_fail(p, LBM_E_INVAL, "invalid argument");
    if (params->storage != p->storage) return pool_fail(p, LBM_E_INVAL, "storage differs from the pool's");
    if (params->root_finder != 0) return pool_fail(p, LBM_E_INVAL, "the pool runs the Newton root finder only");
    if ((int64_t)params->nx * params->ny * params->nz >= kWideCells)
        return pool_fail(p, LBM_E_INVAL, "pool slots take fewer than 2^28 cells");
    const int64_t need = lbm_required_bytes(params);
    if (need < 0) return pool_fail(p, (int)need, lbm_last_error(nullptr));
    int slot = -1;
    for (int i = 0; i < p->max_slots; ++i)
        if (!p->slots[i].used) {
            slot = i;
            break;
        }
    if (slot < 0) return pool_fail(p, LBM_E_NOMEM, "no free slot");
    const int64_t off = p->heap.alloc(need);
    if (off < 0) return pool_fail(p, LBM_E_NOMEM, "no free range of " + std::to_string(need) + " bytes");
    // created on the admission stream: overlaps a round in flight, whose
    // slots own disjoint arena ranges
    lbm_ctx *ctx = nullptr;
    const int rc = lbm_create(params, p->arena + off, need, p->admit_stream, &ctx);
    if (rc != LBM_OK) {
        p->heap.release(off, need);
        return pool_fail(p, rc, lbm_last_error(nullptr));
    }
    const hipError_t e = hipEventRecord(p->admitted, p->admit_stream);
    if (e != hipSuccess) {
        (void)lbm_destroy(ctx);
        p->heap.release(off, need);
        return pool_fail(p, LBM_E_DEVICE, std::string("admission event: ") + hipGetErrorString(e));
    }
    PoolSlot &s = p->slots[slot];
    s.used = true;
    s.in_round = false;
    s.ctx = ctx;
    s.off = off;
    s.bytes = need;
    s.steps_total = nsteps;
    s.steps_left = nsteps;
    s.admitted_seq = p->seq++;
    s.admitted_at = host_seconds();
    *slot_out = slot;
    return LBM_OK;
}

int lbm_pool_launch(lbm_pool *p, int32_t *nlaunched)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "pool is NULL");
    if (nlaunched) *nlaunched = 0;
    if (p->in_flight) return pool_fail(p, LBM_E_INVAL, "a round is already in flight");
    const std::vector<int> run = pick_round(p);
    if (run.empty()) return LBM_OK;
    SlotTable *t = p->h_table;
    int blocks = 0, n = 0;
    for (int i : run) {
        PoolSlot &s = p->slots[i];
        SlotDesc d = s.ctx->desc;
        d.parity0 = (int32_t)(s.ctx->steps & 1);
        d.steps_todo = (int32_t)std::min<int64_t>(p->graph_steps, s.steps_left);
        d.stats = nullptr;
        t->slot[n] = d;
        t->block_start[n] = blocks;
        blocks += d.blocks;
        ++n;
    }
    t->nslots = n;
    t->block_start[n] = blocks;
    t->total_blocks = blocks;
    POOL_TRY(p, hipStreamWaitEvent(p->stream, p->admitted, 0));
    POOL_TRY(p, hipMemcpyAsync(p->d_table, t, slot_table_bytes(n), hipMemcpyHostToDevice, p->stream));
    POOL_TRY(p, hipGraphLaunch(p->exec, p->stream));
    for (int i : run) p->slots[i].in_round = true;
    p->round = run;
    p->in_flight = true;
    p->launched_at = host_seconds();
    if (nlaunched) *nlaunched = n;
    return LBM_OK;
}

int lbm_pool_wait(lbm_pool *p, int32_t *finished, int32_t *nfinished)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "pool is NULL");
    if (nfinished) *nfinished = 0;
    if (!p->in_flight) return LBM_OK;
    const hipError_t e = hipStreamSynchronize(p->stream);
    const double dt = host_seconds() - p->launched_at;
    p->in_flight = false;
    int nf = 0;
    double done = 0.0;
    for (int i : p->round) {
        PoolSlot &s = p->slots[i];
        s.in_round = false;
        if (e != hipSuccess) continue;
        const int64_t adv = std::min<int64_t>(p->graph_steps, s.steps_left);
        done += (double)s.ctx->fluid_cells * (double)adv;
        s.ctx->steps += adv;
        s.steps_left -= adv;
        if (s.steps_left == 0) {
            if (finished) finished[nf] = i;
            ++nf;
        }
    }
    p->round.clear();
    // throughput of rounds that fill the device (small rounds are launch-bound)
    if (e == hipSuccess && dt > 0.0 && done >= (double)p->fill_cells * p->graph_steps)
        p->rate = 0.7 * p->rate + 0.3 * (done / dt);
    if (e != hipSuccess) return pool_fail(p, LBM_E_DEVICE, std::string("round failed: ") + hipGetErrorString(e));
    if (nfinished) *nfinished = nf;
    return LBM_OK;
}

int lbm_pool_run(lbm_pool *p, int32_t *finished, int32_t *nfinished)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "pool is NULL");
    if (nfinished) *nfinished = 0;
    const int rc = lbm_pool_launch(p, nullptr);
    if (rc != LBM_OK) return rc;
    return lbm_pool_wait(p, finished, nfinished);
}

int lbm_pool_slot_progress(const lbm_pool *p, int32_t slot, int64_t *steps_done, int64_t *steps_left)
{
    if (!slot_ok(p, slot)) return slot_fail(p);
    if (steps_done) *steps_done = p->slots[slot].steps_total - p->slots[slot].steps_left;
    if (steps_left) *steps_left = p->slots[slot].steps_left;
    return LBM_OK;
}

int lbm_pool_moments(lbm_pool *p, int32_t slot, double *out_host, double *totals)
{
    if (!slot_ok(p, slot)) return slot_fail(p);
    if (p->slots[slot].in_round) return pool_fail(p, LBM_E_INVAL, "slot is part of the round in flight");
    const int rc = lbm_moments(p->slots[slot].ctx, out_host, totals);
    if (rc != LBM_OK) p->err = lbm_last_error(p->slots[slot].ctx);
    return rc;
}

int lbm_pool_release(lbm_pool *p, int32_t slot)
{
    if (!slot_ok(p, slot)) return slot_fail(p);
    if (p->slots[slot].in_round) return pool_fail(p, LBM_E_INVAL, "slot is part of the round in flight");
    PoolSlot &s = p->slots[slot];
    const int rc = lbm_destroy(s.ctx);
    p->heap.release(s.off, s.bytes);
    s = PoolSlot();
    if (rc != LBM_OK) return pool_fail(p, rc, lbm_last_error(nullptr));
    return LBM_OK;
}

int lbm_pool_get_info(const lbm_pool *p, lbm_pool_info *info)
{
    if (!p || !info) return fail(nullptr, LBM_E_INVAL, "pool or info is NULL");
    info->max_slots = p->max_slots;
    info->active = 0;
    info->running = 0;
    for (auto &s : p->slots) {
        info->active += s.used;
        info->running += s.used && s.steps_left > 0;
    }
    info->graph_steps = p->graph_steps;
    info->sched = p->sched;
    info->in_flight = p->in_flight;
    info->fill_cells = p->fill_cells;
    info->arena_bytes = p->arena_bytes;
    info->free_bytes = p->heap.total();
    info->largest_free = p->heap.largest();
    return LBM_OK;
}

int lbm_pool_destroy(lbm_pool *p)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "pool is NULL");
    pool_free(p);
    return LBM_OK;
}

const char *lbm_pool_last_error(const lbm_pool *p) { return p ? p->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
