// Host runtime and C ABI of the gfx950 Vlasov solver (include/vlasov.h).
//
// A context owns no device memory: f (two ping-pong buffers) and the
// workspace are caller allocations.  Host code builds the line tables of the
// x drift (constant over a run) and the model tables (sin/cos of the angle
// nodes, ring-potential derivative and value) with the host libm and uploads
// them once; no transcendental function is evaluated on the device.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "vlasov_internal.hpp"

using namespace vlasov_detail;

namespace {
thread_local std::string g_err;
}

// Workspace of the contexts made by vlasov_init_static, for callers that
// cannot allocate device memory.  Each device the library runs on holds its
// own copy until the process ends.  Host code never passes the name of the
// array to a kernel or a copy (there it is a host-side stand-in): the device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is used.
constexpr size_t STATIC_WS_MAX = (size_t)16 << 20;
static __device__ __align__(256) char scratch[STATIC_WS_MAX];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[STATIC_MAX_DEVICES];   // device address of `scratch` per device
bool g_static_busy[STATIC_MAX_DEVICES];   // a live context holds that device's copy
}  // namespace

namespace vlasov_detail {

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// Substep sizes of the splittings, the doubles nearest to the exact values:
// triple jump w1 = 1/(2 - 2^(1/3)), w0 = -2^(1/3)/(2 - 2^(1/3)); Suzuki
// p = 1/(4 - 4^(1/3)) and 1 - 4p.
int split_weights(int scheme, double *w)
{
    if (scheme == VLASOV_SPLIT_TRIPLE_JUMP) {
        w[0] = w[2] = 1.3512071919596575;
        w[1] = -1.7024143839193153;
        return 3;
    }
    if (scheme == VLASOV_SPLIT_SUZUKI) {
        w[0] = w[1] = w[3] = w[4] = 0.4144907717943757;
        w[2] = -0.657963087177503;
        return 5;
    }
    w[0] = 1.0;
    return 1;
}

Layout layout_of(const vlasov_params &p)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align_up(bytes > 0 ? bytes : 1);
        return at;
    };
    const size_t nx = (size_t)p.nx, np = (size_t)p.np;
    double w[MAX_SUB];
    const size_t ns = (size_t)split_weights(p.splitting, w);
    L.drift_m = take(ns * np * sizeof(int32_t));
    L.drift_w = take(ns * np * sizeof(double4));
    L.kd_base = take(ns * (size_t)nblocks(p.np) * sizeof(int32_t));
    L.kd_rel = take(ns * np * sizeof(int32_t));
    L.part = take((size_t)nblocks(p.np) * nx * sizeof(double));
    L.rho = take(nx * sizeof(double));
    L.F = take(nx * sizeof(double));
    L.Fext = take(nx * sizeof(double));
    L.cs = take(nx * sizeof(double));
    L.sn = take(nx * sizeof(double));
    L.ringK = take(nx * sizeof(double));
    L.ringV = take(nx * sizeof(double));
    L.mxmy = take(2 * sizeof(double));
    L.hist = take((size_t)p.hist_cap * 2 * sizeof(double));
    L.hcount = take(sizeof(int64_t));
    L.mom_out = take(10 * sizeof(double));
    L.mom_col = take(6 * nx * sizeof(double));
    L.mom_phi = take(nx * sizeof(double));
    L.gs_g = take(2 * sizeof(double));
    L.total = o;
    return L;
}

std::string validate(const vlasov_params *p)
{
    if (!p) return "params is NULL";
    if (p->model < 0 || p->model > 3) return "unknown model";
    if (p->storage != VLASOV_F64 && p->storage != VLASOV_F32) return "unknown storage";
    if ((p->bc_x != 0 && p->bc_x != 1) || (p->bc_p != 0 && p->bc_p != 1)) return "unknown boundary";
    if (p->nx < 16 || p->np < 16) return "nx and np must be >= 16";
    // grid.y of the row-block launches is ceil(np/16) <= 65535
    if (p->nx > (1 << 19) || p->np > (1 << 19) || p->nx * p->np >= ((int64_t)1 << 31)) return "grid too large";
    if (!(isfinite(p->xmin) && isfinite(p->xmax) && p->xmax > p->xmin)) return "bad x domain";
    if (!(isfinite(p->pmin) && isfinite(p->pmax) && p->pmax > p->pmin)) return "bad p domain";
    if (!isfinite(p->dt) || p->dt == 0.0) return "dt must be finite and nonzero";
    if ((p->model == VLASOV_MODEL_HMF || p->model == VLASOV_MODEL_RING) && p->bc_x != VLASOV_BC_PERIODIC)
        return "HMF and ring models need a periodic x axis";
    if (p->model == VLASOV_MODEL_RING && !(isfinite(p->ring_eps) && p->ring_eps > 0.0)) return "ring_eps must be > 0";
    if (p->model == VLASOV_MODEL_SHEET && !isfinite(p->sheet_G)) return "sheet_G must be finite";
    if (p->hist_cap < 0) return "hist_cap must be >= 0";
    if (p->spline != VLASOV_SPLINE_FD && p->spline != VLASOV_SPLINE_GS) return "unknown spline";
    if (p->spline == VLASOV_SPLINE_GS && (p->nx > vk::GS_MAX_N || p->np > vk::GS_MAX_N))
        return "the global spline takes lines of at most 4096 samples";
    if (p->splitting < VLASOV_SPLIT_STRANG || p->splitting > VLASOV_SPLIT_SUZUKI) return "unknown splitting";
    if (p->filter_every < 0) return "filter_every must be >= 0";
    if (p->filter_every > 0 && !(isfinite(p->filter_strength) && p->filter_strength > 0.0 && p->filter_strength <= 1.0))
        return "filter_strength must lie in (0, 1]";
    if (p->reserved != 0) return "reserved must be 0";
    return "";
}

}  // namespace vlasov_detail

namespace {

int gs_drift(vlasov_ctx *c, int table, bool partials);
int gs_kick(vlasov_ctx *c, double h);

// The half drift of table ta, then (tb >= 0) that of table tb, in one pass.
int drift(vlasov_ctx *c, int ta, int tb, bool partials)
{
    if (c->P.spline == VLASOV_SPLINE_GS) {  // two half drifts are two passes
        int rc = gs_drift(c, ta, partials && tb < 0);
        if (rc == VLASOV_OK && tb >= 0) rc = gs_drift(c, tb, partials);
        return rc;
    }
    return c->P.storage == VLASOV_F32 ? launch_drift<float>(c, ta, tb, partials)
                                      : launch_drift<double>(c, ta, tb, partials);
}

// Density from the partial sums, then the model force (and magnetization).
int density_force(vlasov_ctx *c)
{
    const vlasov_params &P = c->P;
    const int nx = (int)P.nx;
    double *rho = c->at<double>(c->L.rho);
    double *F = c->at<double>(c->L.F);
    launch(c, VLASOV_K_DENSITY, vk::k_density, dim3((unsigned)((nx + 15) / 16)), dim3(1024),
           c->at<double>(c->L.part), rho, nx, (int)c->nblk, c->dp);
    int rc = check_launch("density");
    if (rc) return rc;
    double *hist = c->at<double>(c->L.hist);
    int64_t *hcount = c->at<int64_t>(c->L.hcount);
    double *mxmy = c->at<double>(c->L.mxmy);
    const double *cs = c->at<double>(c->L.cs), *sn = c->at<double>(c->L.sn);
    switch (P.model) {
    case VLASOV_MODEL_HMF:
        launch(c, VLASOV_K_FORCE, vk::k_force_hmf, dim3(1), dim3(1024), rho, cs, sn, F, nx, c->dx, mxmy, hist, hcount,
               P.hist_cap);
        break;
    case VLASOV_MODEL_RING: {
        const int per = vk::ring_outputs_per_wg(nx);
        launch(c, VLASOV_K_FORCE, nx <= vk::RING_LDS_MAX ? vk::k_force_ring<true> : vk::k_force_ring<false>,
               dim3((unsigned)(1 + (nx + per - 1) / per)), dim3(256), rho, c->at<double>(c->L.ringK), F, nx, c->dx,
               cs, sn, mxmy, hist, hcount, P.hist_cap);
        break;
    }
    case VLASOV_MODEL_SHEET: {
        const double K = ((2.0 * M_PI) * P.sheet_G) * c->dx;
        launch(c, VLASOV_K_FORCE, nx <= vk::SHEET_LDS_MAX ? vk::k_force_sheet<true> : vk::k_force_sheet<false>,
               dim3(1), dim3(1024), rho, F, nx, K);
        break;
    }
    default:
        break;  // EXTERNAL: the kick reads the caller's force table
    }
    rc = check_launch("force");
    if (rc == VLASOV_OK) c->have_force = true;
    return rc;
}

int kick(vlasov_ctx *c, double h)
{
    if (c->P.spline == VLASOV_SPLINE_GS) return gs_kick(c, h);
    return c->P.storage == VLASOV_F32 ? launch_kick<float>(c, h) : launch_kick<double>(c, h);
}

// The filter along p with strength sigma = filter_strength.
int filter(vlasov_ctx *c)
{
    return c->P.storage == VLASOV_F32 ? launch_filter<float>(c) : launch_filter<double>(c);
}

// Kick of step size h and the filter in one pass (local spline).
int kick_filter(vlasov_ctx *c, double h)
{
    if (c->P.spline == VLASOV_SPLINE_GS) {
        int rc = kick(c, h);
        return rc == VLASOV_OK ? filter(c) : rc;
    }
    return c->P.storage == VLASOV_F32 ? launch_kick_filter<float>(c, h) : launch_kick_filter<double>(c, h);
}

// ---------------------------------------------------------------------------
// Global spline (eq. tridiagsys): one workgroup per line; the kick runs on the
// rows of the transpose.
// ---------------------------------------------------------------------------
int gs_drift(vlasov_ctx *c, int table, bool partials)
{
    return c->P.storage == VLASOV_F32 ? gs_drift_t<float>(c, table, partials) : gs_drift_t<double>(c, table, partials);
}

int gs_kick(vlasov_ctx *c, double h)
{
    return c->P.storage == VLASOV_F32 ? gs_kick_t<float>(c, h) : gs_kick_t<double>(c, h);
}

// Fused kick and two half drifts (+ density partial sums) on tiles of TW
// columns by RB density blocks.
int kick_then_drift(vlasov_ctx *c, int k, int tb, double h, bool filt)
{
    const int w = c->tune.kick_drift_width;
    if (tb >= 0 && !filt && w != 0 && c->kd_ok[k] && c->P.spline == VLASOV_SPLINE_FD) {
        const bool f32 = c->P.storage == VLASOV_F32;
        if (w == 230) return f32 ? launch_kick_drift_w<float, 230>(c, k, h) : launch_kick_drift_w<double, 230>(c, k, h);
        return f32 ? launch_kick_drift_w<float, 486>(c, k, h) : launch_kick_drift_w<double, 486>(c, k, h);
    }
    int rc = filt ? kick_filter(c, h) : kick(c, h);
    if (rc == VLASOV_OK) rc = drift(c, k, tb, tb >= 0);
    return rc;
}

// Tables of the fused kick and drift for tiles of rb density blocks, one set
// per pair (k, k + 1 mod nsub) of drift tables: row j's two half drifts move
// its window by o_j = m_k,j + m_k+1,j columns; per tile the start of its
// kicked column range relative to the tile, per row the offset of its window
// in that range.  Sets kd_ok[k] (the single-grid kernels' slack) and
// kd_spread[k]; the tables are filled for spreads up to the batched kernel's
// wider slack.
void build_kd_tables(vlasov_ctx *c, int rb)
{
    const vlasov_params &P = c->P;
    const int64_t rows = (int64_t)vk::ROWS_PER_BLOCK * rb, ntile = (c->nblk + rb - 1) / rb;
    c->h_kd_base.assign((size_t)c->nsub * (size_t)c->nblk, 0);
    c->h_kd_rel.assign((size_t)c->nsub * (size_t)P.np, 0);
    for (int k = 0; k < c->nsub; ++k) {
        const int64_t *ma = c->h_mfull.data() + (size_t)k * (size_t)P.np;
        const int64_t *mb = c->h_mfull.data() + (size_t)((k + 1) % c->nsub) * (size_t)P.np;
        int32_t *base = c->h_kd_base.data() + (size_t)k * (size_t)c->nblk;
        int32_t *rel = c->h_kd_rel.data() + (size_t)k * (size_t)P.np;
        int64_t spread = 0;
        for (int64_t b = 0; b < ntile; ++b) {
            const int64_t j0 = b * rows, j1 = std::min<int64_t>(P.np, j0 + rows);
            int64_t lo = ma[j0] + mb[j0], hi = lo;
            for (int64_t j = j0; j < j1; ++j) {
                lo = std::min(lo, ma[j] + mb[j]);
                hi = std::max(hi, ma[j] + mb[j]);
            }
            spread = std::max(spread, hi - lo);
            if (hi - lo > vk::KD_SPR_WIDE) continue;  // not fusable; the tables are unused
            for (int64_t j = j0; j < j1; ++j) rel[j] = (int32_t)(ma[j] + mb[j] - lo);
            int64_t s0 = lo - 8;
            if (P.bc_x == VLASOV_BC_PERIODIC) {
                s0 %= P.nx;
                if (s0 < 0) s0 += P.nx;
            }
            base[b] = (int32_t)s0;
        }
        c->kd_ok[k] = spread <= vk::KD_SPR;
        c->kd_spread[k] = spread;
    }
    c->kd_rb = rb;
}

int upload_kd_tables(vlasov_ctx *c)
{
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.kd_base, c->h_kd_base.data(), c->h_kd_base.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.kd_rel, c->h_kd_rel.data(), c->h_kd_rel.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return VLASOV_OK;
}

void to_host_f(const vlasov_ctx *c, const void *src, double *dst)
{
    const size_t N = (size_t)c->P.nx * (size_t)c->P.np;
    if (c->P.storage == VLASOV_F32) {
        const float *s = (const float *)src;
        for (size_t k = 0; k < N; ++k) dst[k] = (double)s[k];
    } else {
        memcpy(dst, src, N * sizeof(double));
    }
}

int upload_f(vlasov_ctx *c, const double *f_host)
{
    const size_t N = (size_t)c->P.nx * (size_t)c->P.np;
    if (c->P.storage == VLASOV_F32) {
        std::vector<float> tmp(N);
        for (size_t k = 0; k < N; ++k) tmp[k] = (float)f_host[k];
        HIP_TRY(hipMemcpyAsync(c->fcur(), tmp.data(), N * sizeof(float), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
        HIP_TRY(hipMemcpyAsync(c->fcur(), f_host, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return VLASOV_OK;
}

// Steps 2-4 of one (sub)step sequence and step 1 of the next: the body of a
// step that is not the last of a call (more = true), or of the last one.
int step_body(vlasov_ctx *c, bool more)
{
    const int every = c->P.filter_every;
    const bool filtered = every > 0 && (c->steps_done + 1) % every == 0;
    int rc = VLASOV_OK;
    for (int k = 0; rc == VLASOV_OK && k < c->nsub; ++k) {
        rc = density_force(c);  // step 2
        // step 3 (+ the filter after the last kick of a filtered step),
        // step 4, and step 1 of the next substep (or step)
        const bool last = k + 1 == c->nsub;
        const int tb = !last ? k + 1 : (more ? 0 : -1);
        if (rc == VLASOV_OK) rc = kick_then_drift(c, k, tb, c->wsub[k] * c->P.dt, filtered && last);
    }
    if (rc == VLASOV_OK) ++c->steps_done;
    return rc;
}

void drop_graphs(vlasov_ctx *c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        c->gexec[k] = nullptr;
    }
}

// gsteps steps that are not the last of a call, as one graph launch: the
// graph for the current buffer is captured (on a private stream; the host
// state advances as the capture enqueues) and then replayed with the host
// state advanced by hand.  The sequence of kernels of such a step depends
// only on the current buffer (no filter schedule: graphs are not used with
// the filter).
int graph_steps(vlasov_ctx *c)
{
    const int start = c->cur;
    if (!c->gexec[start]) {
        if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        int rc = e == hipSuccess ? VLASOV_OK : fail(VLASOV_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        const int64_t done0 = c->steps_done;
        for (int s = 0; rc == VLASOV_OK && s < c->gsteps; ++s) rc = step_body(c, true);
        hipGraph_t g = nullptr;
        if (e == hipSuccess) e = hipStreamEndCapture(c->cap_stream, &g);
        c->stream = user;
        c->steps_done = done0;
        if (rc == VLASOV_OK && e != hipSuccess) rc = fail(VLASOV_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        if (rc == VLASOV_OK) {
            e = hipGraphInstantiate(&c->gexec[start], g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                c->gexec[start] = nullptr;
                rc = fail(VLASOV_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
        }
        if (g) (void)hipGraphDestroy(g);
        if (rc != VLASOV_OK) return rc;
        c->gcur_end[start] = c->cur;
    }
    HIP_TRY(hipGraphLaunch(c->gexec[start], c->stream));
    c->cur = c->gcur_end[start];
    c->have_force = true;
    c->steps_done += c->gsteps;
    return VLASOV_OK;
}

}  // namespace

extern "C" {

const char *vlasov_last_error(void) { return g_err.c_str(); }

size_t vlasov_f_bytes(const vlasov_params *p)
{
    if (!validate(p).empty()) return 0;
    return 2 * (size_t)p->nx * (size_t)p->np * (p->storage == VLASOV_F32 ? 4 : 8);
}

size_t vlasov_workspace_bytes(const vlasov_params *p)
{
    if (!validate(p).empty()) return 0;
    return layout_of(*p).total;
}

int vlasov_init(const vlasov_params *p, const double *f0_host, void *f_dev, void *ws_dev, void *hip_stream,
                vlasov_ctx **out)
{
    std::string why = validate(p);
    if (!why.empty()) return fail(VLASOV_E_INVAL, why);
    if (!f_dev || !ws_dev || !out) return fail(VLASOV_E_INVAL, "NULL pointer argument");
    if (((uintptr_t)f_dev % ALIGN) || ((uintptr_t)ws_dev % ALIGN))
        return fail(VLASOV_E_INVAL, "device buffers must be 256-byte aligned");
    vlasov_ctx *c = new vlasov_ctx();
    c->P = *p;
    c->stream = (hipStream_t)hip_stream;
    c->s = p->storage == VLASOV_F32 ? 4 : 8;
    const size_t N = (size_t)p->nx * (size_t)p->np;
    c->f[0] = (char *)f_dev;
    c->f[1] = (char *)f_dev + N * c->s;
    c->cur = 0;
    c->ws = (char *)ws_dev;
    c->L = layout_of(*p);
    c->dx = (p->xmax - p->xmin) / (double)p->nx;
    c->dp = (p->pmax - p->pmin) / (double)p->np;
    c->nblk = nblocks(p->np);
    c->have_force = false;
    c->prof = false;
    c->tune.drift_threads = DRIFT_NT;
    c->tune.kick_rows = p->storage == VLASOV_F32 ? kick_rows<float>() : kick_rows<double>();
    c->tune.kick_drift_width = KD_TW;
    c->tune.kick_drift_blocks = default_kd_blocks(p->nx, c->nblk);
    for (int k = 0; k < VLASOV_K_COUNT; ++k) {
        c->ms[k] = 0.0;
        c->cnt[k] = 0;
    }

    // Drift line tables (eqs. step1, step4), one per substep k: row j moves
    // by p_j tau_k / dx with tau_k = (w_k dt)/2 (dt/2 for the Strang step).
    c->nsub = split_weights(p->splitting, c->wsub);
    c->steps_done = 0;
    const size_t ntab = (size_t)c->nsub * (size_t)p->np;
    c->h_dm.resize(ntab);
    c->h_dw.resize(ntab);
    c->h_mfull.resize(ntab);
    for (int k = 0; k < c->nsub; ++k) {
        const double tau = 0.5 * (c->wsub[k] * p->dt);
        for (int64_t j = 0; j < p->np; ++j) {
            const size_t e = (size_t)k * (size_t)p->np + (size_t)j;
            const double pj = p->pmin + (double)j * c->dp;
            const vk::Foot ft = vk::foot_of_shift((pj * tau) / c->dx);
            c->h_dm[e] = vk::reduce_offset(ft.m, p->nx, p->bc_x);
            c->h_dw[e] = make_double4(ft.a, ft.b, ft.g, ft.d);
            // offsets as the drift uses them: the exact foot on a periodic axis
            // (the windows of a tile are then one contiguous range mod nx), the
            // clamped one with zero extension
            c->h_mfull[e] = p->bc_x == VLASOV_BC_PERIODIC ? ft.m : (int64_t)c->h_dm[e];
        }
    }
    build_kd_tables(c, c->tune.kick_drift_blocks);
    // Model tables.
    std::vector<double> cs((size_t)p->nx), sn((size_t)p->nx), K((size_t)p->nx, 0.0), V((size_t)p->nx, 0.0);
    for (int64_t i = 0; i < p->nx; ++i) {
        const double th = p->xmin + (double)i * c->dx;
        cs[i] = cos(th);
        sn[i] = sin(th);
    }
    if (p->model == VLASOV_MODEL_RING) {
        // eq. (ringpot): V(d) = -1/sqrt(q), V'(d) = sin d / (q sqrt q),
        // q = 2 (1 + eps - cos d); V' made exactly odd, V exactly even.
        const int64_t n = p->nx;
        auto dV = [&](double d) {
            const double q = 2.0 * ((1.0 + p->ring_eps) - cos(d));
            return sin(d) / (q * sqrt(q));
        };
        auto Vd = [&](double d) {
            const double q = 2.0 * ((1.0 + p->ring_eps) - cos(d));
            return -1.0 / sqrt(q);
        };
        for (int64_t s = 0; s < n; ++s) {
            if (s == 0 || 2 * s == n)
                K[s] = 0.0;
            else if (2 * s < n)
                K[s] = dV((double)s * c->dx);
            else
                K[s] = -dV((double)(n - s) * c->dx);
            const int64_t e = (2 * s > n) ? n - s : s;
            V[s] = Vd((double)e * c->dx);
        }
    }
    // Recursion coefficients of the (1, 4, 1) operator of eq. (tridiagsys):
    // its root r = sqrt(3) - 2 and the factor -6 r of D
    std::vector<double> gs(2);
    gs[0] = sqrt(3.0) - 2.0;
    gs[1] = -6.0 * gs[0];
    const size_t nxb = (size_t)p->nx * sizeof(double);
    auto cleanup_fail = [&](int rc) {
        delete c;
        return rc;
    };
    int rc = VLASOV_OK;
    const struct {
        size_t off;
        const void *src;
        size_t bytes;
    } ups[] = {{c->L.drift_m, c->h_dm.data(), ntab * sizeof(int32_t)},
               {c->L.drift_w, c->h_dw.data(), ntab * sizeof(double4)},
               {c->L.kd_base, c->h_kd_base.data(), c->h_kd_base.size() * sizeof(int32_t)},
               {c->L.kd_rel, c->h_kd_rel.data(), c->h_kd_rel.size() * sizeof(int32_t)},
               {c->L.cs, cs.data(), nxb},
               {c->L.sn, sn.data(), nxb},
               {c->L.ringK, K.data(), nxb},
               {c->L.ringV, V.data(), nxb},
               {c->L.gs_g, gs.data(), gs.size() * sizeof(double)}};
    for (const auto &u : ups) {
        hipError_t e = hipMemcpyAsync(c->ws + u.off, u.src, u.bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return cleanup_fail(fail(VLASOV_E_HIP, std::string("table upload: ") + hipGetErrorString(e)));
    }
    if (hipMemsetAsync(c->ws + c->L.Fext, 0, nxb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ws + c->L.hcount, 0, sizeof(int64_t), c->stream) != hipSuccess ||
        hipMemsetAsync(c->ws + c->L.mxmy, 0, 2 * sizeof(double), c->stream) != hipSuccess)
        return cleanup_fail(fail(VLASOV_E_HIP, "workspace clear failed"));
    if (f0_host) {
        if ((rc = upload_f(c, f0_host)) != VLASOV_OK) return cleanup_fail(rc);
    } else if (hipStreamSynchronize(c->stream) != hipSuccess) {  // the host tables above are locals
        return cleanup_fail(fail(VLASOV_E_HIP, "table upload failed"));
    }
    *out = c;
    return VLASOV_OK;
}

int vlasov_init_static(const vlasov_params *p, const double *f0_host, void *f_dev, void *hip_stream,
                       vlasov_ctx **out)
{
    std::string why = validate(p);
    if (!why.empty()) return fail(VLASOV_E_INVAL, why);
    if (!f_dev || !out) return fail(VLASOV_E_INVAL, "NULL pointer argument");
    const size_t wb = layout_of(*p).total;
    if (wb > STATIC_WS_MAX)
        return fail(VLASOV_E_INVAL, "workspace of " + std::to_string(wb) + " bytes exceeds the static maximum of " +
                                        std::to_string(STATIC_WS_MAX) + " bytes (use vlasov_init)");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(VLASOV_E_INVAL, "device ordinal out of range");
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, f_dev) != hipSuccess || attr.device != dev) {
        (void)hipGetLastError();
        return fail(VLASOV_E_INVAL, "f_dev is not device memory of the current device");
    }
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_busy[dev])
            return fail(VLASOV_E_STATE, "the static workspace of device " + std::to_string(dev) +
                                            " is held by a live context (destroy it first)");
        if (!g_static_ptr[dev]) {
            void *ptr = nullptr;
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(VLASOV_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            g_static_ptr[dev] = ptr;
        }
        ws = g_static_ptr[dev];
        g_static_busy[dev] = true;
    }
    const int rc = vlasov_init(p, f0_host, f_dev, ws, hip_stream, out);
    if (rc != VLASOV_OK) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[dev] = false;
        return rc;
    }
    (*out)->static_dev = dev;
    return VLASOV_OK;
}

int vlasov_set_external_force(vlasov_ctx *c, const double *F_host)
{
    if (!c || !F_host) return fail(VLASOV_E_INVAL, "NULL argument");
    if (c->P.model != VLASOV_MODEL_EXTERNAL) return fail(VLASOV_E_STATE, "not an EXTERNAL-force context");
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.Fext, F_host, (size_t)c->P.nx * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return VLASOV_OK;
}

int vlasov_step(vlasov_ctx *c, int64_t nsteps)
{
    if (!c) return fail(VLASOV_E_INVAL, "NULL context");
    if (nsteps < 0) return fail(VLASOV_E_INVAL, "nsteps must be >= 0");
    if (nsteps == 0) return VLASOV_OK;
    int rc = drift(c, 0, -1, true);  // step 1 of the first (sub)step
    int64_t s = 0;
    // steps before the last one, gsteps at a time from a graph (not while
    // per-kernel timers are on, nor with the filter, whose schedule depends
    // on the step count)
    const bool graphs = c->gsteps > 0 && !c->prof && c->P.filter_every == 0;
    while (graphs && rc == VLASOV_OK && nsteps - 1 - s >= c->gsteps) {
        rc = graph_steps(c);
        s += c->gsteps;
    }
    for (; rc == VLASOV_OK && s < nsteps; ++s) rc = step_body(c, s + 1 < nsteps);
    return rc;
}

int vlasov_set_graph(vlasov_ctx *c, int32_t steps_per_graph)
{
    if (!c) return fail(VLASOV_E_INVAL, "NULL context");
    if (steps_per_graph < 0 || steps_per_graph > 4096) return fail(VLASOV_E_INVAL, "steps_per_graph must be in [0, 4096]");
    if (steps_per_graph != c->gsteps) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        drop_graphs(c);
        c->gsteps = steps_per_graph;
    }
    return VLASOV_OK;
}

int vlasov_drift(vlasov_ctx *c, int32_t npass)
{
    if (!c) return fail(VLASOV_E_INVAL, "NULL context");
    if (npass != 1 && npass != 2) return fail(VLASOV_E_INVAL, "npass must be 1 or 2");
    return drift(c, 0, npass == 2 ? 0 : -1, true);
}

int vlasov_force(vlasov_ctx *c, double *F_host, double *mxmy_host)
{
    if (!c) return fail(VLASOV_E_INVAL, "NULL context");
    // density partial sums of the current f: reuse the diagnostic block pass
    const vlasov_params &P = c->P;
    dim3 grid((unsigned)((P.nx + 255) / 256), (unsigned)c->nblk);
    double *scratch = (double *)c->fnext();
    if (P.storage == VLASOV_F32)
        vk::k_mom_blocks<float><<<grid, 256, 0, c->stream>>>((const float *)c->fcur(), scratch, (int)P.nx, (int)P.np,
                                                             (int)c->nblk, P.pmin, c->dp);
    else
        vk::k_mom_blocks<double><<<grid, 256, 0, c->stream>>>((const double *)c->fcur(), scratch, (int)P.nx,
                                                              (int)P.np, (int)c->nblk, P.pmin, c->dp);
    int rc = check_launch("force: block sums");
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.part, scratch, (size_t)c->nblk * (size_t)P.nx * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream));
    if ((rc = density_force(c)) != VLASOV_OK) return rc;
    if (F_host || mxmy_host) {
        if (F_host)
            HIP_TRY(hipMemcpyAsync(F_host, force_ptr(c), (size_t)P.nx * sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream));
        double mm[2] = {0.0, 0.0};
        if (mxmy_host && (P.model == VLASOV_MODEL_HMF || P.model == VLASOV_MODEL_RING))
            HIP_TRY(hipMemcpyAsync(mm, c->ws + c->L.mxmy, sizeof mm, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (mxmy_host) {
            mxmy_host[0] = mm[0];
            mxmy_host[1] = mm[1];
        }
    }
    return VLASOV_OK;
}

int vlasov_kick(vlasov_ctx *c)
{
    if (!c) return fail(VLASOV_E_INVAL, "NULL context");
    if (!c->have_force) return fail(VLASOV_E_STATE, "no force computed yet");
    return kick(c, c->wsub[0] * c->P.dt);
}

int vlasov_moments(vlasov_ctx *c, vlasov_moments_t *out)
{
    if (!c || !out) return fail(VLASOV_E_INVAL, "NULL argument");
    const vlasov_params &P = c->P;
    const int nx = (int)P.nx;
    double *scratch = (double *)c->fnext();  // the idle buffer of the pair
    double *col = c->at<double>(c->L.mom_col);
    double *phi = c->at<double>(c->L.mom_phi);
    double *res = c->at<double>(c->L.mom_out);
    const dim3 grid((unsigned)((P.nx + 255) / 256), (unsigned)c->nblk);
    if (P.storage == VLASOV_F32)
        launch(c, VLASOV_K_MOMENTS, vk::k_mom_blocks<float>, grid, dim3(256), (const float *)c->fcur(), scratch, nx,
               (int)P.np, (int)c->nblk, P.pmin, c->dp);
    else
        launch(c, VLASOV_K_MOMENTS, vk::k_mom_blocks<double>, grid, dim3(256), (const double *)c->fcur(), scratch, nx,
               (int)P.np, (int)c->nblk, P.pmin, c->dp);
    launch(c, VLASOV_K_MOMENTS, vk::k_mom_cols, dim3((unsigned)((nx + 3) / 4)), dim3(256), scratch, col, nx,
           (int)c->nblk, c->dp, 4, 0);
    // entropy density and negative mass: a second block pass over the scratch
    if (P.storage == VLASOV_F32)
        launch(c, VLASOV_K_MOMENTS, vk::k_mom_blocks2<float>, grid, dim3(256), (const float *)c->fcur(), scratch, nx,
               (int)P.np, (int)c->nblk);
    else
        launch(c, VLASOV_K_MOMENTS, vk::k_mom_blocks2<double>, grid, dim3(256), (const double *)c->fcur(), scratch,
               nx, (int)P.np, (int)c->nblk);
    launch(c, VLASOV_K_MOMENTS, vk::k_mom_cols, dim3((unsigned)((nx + 3) / 4)), dim3(256), scratch, col, nx,
           (int)c->nblk, c->dp, 2, 4);
    double wcoef = 0.0;
    if (P.model == VLASOV_MODEL_RING) {
        launch(c, VLASOV_K_MOMENTS, vk::k_mom_phi<true>, dim3((unsigned)((nx + 3) / 4)), dim3(256), col,
               c->at<double>(c->L.ringV), phi, nx);
        wcoef = (0.5 * c->dx) * c->dx;
    } else if (P.model == VLASOV_MODEL_SHEET) {
        launch(c, VLASOV_K_MOMENTS, vk::k_mom_phi<false>, dim3((unsigned)((nx + 3) / 4)), dim3(256), col,
               (const double *)nullptr, phi, nx);
        wcoef = (((M_PI * P.sheet_G) * c->dx) * c->dx) * c->dx;
    }
    launch(c, VLASOV_K_MOMENTS, vk::k_mom_final, dim3(1), dim3(64), col, phi, c->at<double>(c->L.cs),
           c->at<double>(c->L.sn), res, nx, c->dx, (int)P.model, wcoef);
    int rc = check_launch("moments");
    if (rc) return rc;
    double h[10];
    HIP_TRY(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out->mass = h[0];
    out->momentum = h[1];
    out->kinetic = h[2];
    out->potential = h[3];
    out->energy = h[4];
    out->mx = h[5];
    out->my = h[6];
    out->l2 = h[7];
    out->entropy = h[8];
    out->neg_mass = h[9];
    for (double v : h)
        if (!isfinite(v)) return fail(VLASOV_E_NONFINITE, "non-finite diagnostic");
    return VLASOV_OK;
}

int vlasov_mag_history(vlasov_ctx *c, double *mx, double *my, int64_t cap, int64_t *count)
{
    if (!c || !count || cap < 0 || (cap > 0 && (!mx || !my))) return fail(VLASOV_E_INVAL, "bad argument");
    int64_t n = 0;
    HIP_TRY(hipMemcpyAsync(&n, c->ws + c->L.hcount, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    int64_t k = n < cap ? n : cap;
    if (k > c->P.hist_cap) k = c->P.hist_cap;
    if (k > 0) {
        std::vector<double> h((size_t)k * 2);
        HIP_TRY(hipMemcpyAsync(h.data(), c->ws + c->L.hist, (size_t)k * 2 * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int64_t t = 0; t < k; ++t) {
            mx[t] = h[2 * t];
            my[t] = h[2 * t + 1];
        }
    }
    *count = n;
    return VLASOV_OK;
}

int vlasov_read_f(vlasov_ctx *c, double *f_host)
{
    if (!c || !f_host) return fail(VLASOV_E_INVAL, "NULL argument");
    const size_t bytes = (size_t)c->P.nx * (size_t)c->P.np * c->s;
    std::vector<char> tmp(bytes);
    HIP_TRY(hipMemcpyAsync(tmp.data(), c->fcur(), bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    to_host_f(c, tmp.data(), f_host);
    return VLASOV_OK;
}

int vlasov_write_f(vlasov_ctx *c, const double *f_host)
{
    if (!c || !f_host) return fail(VLASOV_E_INVAL, "NULL argument");
    return upload_f(c, f_host);
}

int vlasov_destroy(vlasov_ctx *c)
{
    if (!c) return VLASOV_OK;
    (void)hipStreamSynchronize(c->stream);
    for (auto &r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[c->static_dev] = false;
    }
    delete c;
    return VLASOV_OK;
}

int vlasov_tuning_candidates(vlasov_tuning *out, int32_t cap, int32_t *n)
{
    static const int nts[] = {64, 128, 256}, rs[] = {8, 16, 32};
    if (!n || cap < 0 || (cap > 0 && !out)) return fail(VLASOV_E_INVAL, "bad argument");
    // the default tile first (ties in a tuner go to the earlier shape)
    static const int kdw[] = {KD_TW, 486}, kdb[] = {KD_RB, 1, 3, 4};
    static_assert(KD_TW == 230 && KD_RB == 2, "candidate lists hold the default once");
    int k = 0;
    for (int a : nts)
        for (int r : rs) {
            if (k < cap) out[k] = vlasov_tuning{a, r, 0, 1};
            ++k;
        }
    // fused kick and drift (the drift and kick shapes serve the first and last
    // half drift of a call and grids that cannot fuse)
    for (int w : kdw)
        for (int b : kdb) {
            if (k < cap) out[k] = vlasov_tuning{DRIFT_NT, kick_rows<double>(), w, b};
            ++k;
        }
    *n = k;
    return VLASOV_OK;
}

int vlasov_set_tuning(vlasov_ctx *c, const vlasov_tuning *t)
{
    if (!c || !t) return fail(VLASOV_E_INVAL, "NULL argument");
    const bool nt_ok = t->drift_threads == 64 || t->drift_threads == 128 || t->drift_threads == 256;
    const bool r_ok = t->kick_rows == 8 || t->kick_rows == 16 || t->kick_rows == 32;
    const bool w_ok = t->kick_drift_width == 0 || t->kick_drift_width == 230 || t->kick_drift_width == 486;
    const bool b_ok = t->kick_drift_blocks >= 1 && t->kick_drift_blocks <= 4;
    if (!nt_ok || !r_ok || !w_ok || !b_ok) return fail(VLASOV_E_INVAL, "launch shape not compiled in");
    const bool retable = t->kick_drift_blocks != c->kd_rb;
    HIP_TRY(hipStreamSynchronize(c->stream));  // the graphs of the old shape may still run
    drop_graphs(c);
    c->tune = *t;
    if (retable) {
        HIP_TRY(hipStreamSynchronize(c->stream));  // no kernel may read the tables being replaced
        build_kd_tables(c, t->kick_drift_blocks);
        return upload_kd_tables(c);
    }
    return VLASOV_OK;
}

int vlasov_get_tuning(vlasov_ctx *c, vlasov_tuning *t)
{
    if (!c || !t) return fail(VLASOV_E_INVAL, "NULL argument");
    *t = c->tune;
    return VLASOV_OK;
}

int vlasov_profile_enable(vlasov_ctx *c, int32_t on)
{
    if (!c) return fail(VLASOV_E_INVAL, "NULL context");
    if (on && !c->prof) {
        for (int k = 0; k < VLASOV_K_COUNT; ++k) {
            c->ms[k] = 0.0;
            c->cnt[k] = 0;
        }
    }
    c->prof = on != 0;
    return VLASOV_OK;
}

int vlasov_profile_read(vlasov_ctx *c, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!c || kernel < 0 || kernel >= VLASOV_K_COUNT) return fail(VLASOV_E_INVAL, "bad argument");
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto &r : c->recs) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        c->ms[r.kid] += ms;
        c->cnt[r.kid] += 1;
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    if (total_ms) *total_ms = c->ms[kernel];
    if (launches) *launches = c->cnt[kernel];
    return VLASOV_OK;
}

const char *vlasov_kernel_name(int32_t kernel)
{
    static const char *names[VLASOV_K_COUNT] = {"drift", "drift2", "density", "force", "kick", "moments", "kick_drift2", "filter"};
    return (kernel >= 0 && kernel < VLASOV_K_COUNT) ? names[kernel] : "";
}

int vlasov_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (!dst || !src || (bytes % 16)) return fail(VLASOV_E_INVAL, "bad copy arguments");
    const size_t n = bytes / 16;
    if (n == 0) return VLASOV_OK;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0xFFFFFFFFull) return fail(VLASOV_E_INVAL, "copy too large");
    vk::k_copy<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>((const double2 *)src, (double2 *)dst, n);
    return check_launch("copy");
}

}  // extern "C"
