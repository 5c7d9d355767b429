// Initial conditions of the paper's workloads (Sec. 4), generated on the
// device into a context's f (vlasov_generate_ic; the server's requests):
// waterbags, with the HMF map from (U, M0) to the half-widths, and the
// homogeneous Gaussian with a cos(x) seed.  Every one is normalised to unit
// mass on the grid with the raw values summed in index order, so that the
// result is a function of the specification alone.
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "vlasov_internal.hpp"

using namespace vlasov_detail;

namespace {

// SplitMix64 (Steele, Lea and Flood 2014), counter-based: output k of the
// stream of `seed`.
constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull, SM_M1 = 0xBF58476D1CE4E5B9ull, SM_M2 = 0x94D049BB133111EBull;

__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * SM_GAMMA;
    z = (z ^ (z >> 30)) * SM_M1;
    z = (z ^ (z >> 27)) * SM_M2;
    return z ^ (z >> 31);
}

// Uniform double in [0, 1) from the top 53 bits.
__host__ __device__ inline double uniform01(uint64_t seed, uint64_t k)
{
    return (double)(splitmix64(seed, k) >> 11) * 0x1p-53;
}

struct Grid {
    int nx, np;
    double xmin, dx, pmin, dp;
};

struct Bag {
    double x0, p0, amp;
    uint64_t seed;
};

__device__ __forceinline__ double waterbag_raw(const Grid &g, const Bag &w, int i, int j)
{
    const double x = g.xmin + (double)i * g.dx;
    const double v = g.pmin + (double)j * g.dp;
    if (!(fabs(v) <= w.p0 && fabs(x) <= w.x0)) return 0.0;
    if (w.amp == 0.0) return 1.0;
    const double eta = 2.0 * uniform01(w.seed, (uint64_t)j * (uint64_t)g.nx + (uint64_t)i) - 1.0;
    return 1.0 + w.amp * eta;
}

// Raw waterbag values, FP64, into `raw` (nx np values).
__global__ void k_ic_bag_raw(double *__restrict__ raw, Grid g, Bag w)
{
    const size_t n = (size_t)g.nx * (size_t)g.np;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        raw[e] = waterbag_raw(g, w, (int)(e % (size_t)g.nx), (int)(e / (size_t)g.nx));
}

// s + a[0] + a[1] + ... + a[n-1], added one by one in index order; sixteen
// terms requested at a time.
__device__ __forceinline__ double serial_sum(const double *__restrict__ a, int n)
{
    double s = 0.0;
    int i = 0;
    for (; i + 16 <= n; i += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = a[i + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) s = s + v[u];
    }
    for (; i < n; ++i) s = s + a[i];
    return s;
}

// Serial sum of each row (one thread per row, from i = 0).
__global__ void k_ic_rows_raw(const double *__restrict__ raw, double *__restrict__ rows, Grid g)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.np) return;
    rows[j] = serial_sum(raw + (size_t)j * (size_t)g.nx, g.nx);
}

__global__ void k_ic_rows_gauss(const double *__restrict__ e, const double *__restrict__ c,
                                double *__restrict__ rows, Grid g)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.np) return;
    const double ej = e[j];
    double s = 0.0;
    for (int i = 0; i < g.nx; ++i) s = s + ej * c[i];
    rows[j] = s;
}

// The serial sum of the row sums S and the divisor (S dx) dp.
__global__ void k_ic_norm(const double *__restrict__ rows, double *__restrict__ norm, Grid g)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double s = serial_sum(rows, g.np);
    norm[0] = (s * g.dx) * g.dp;
}

template <typename T>
__global__ void k_ic_bag_fill(T *__restrict__ f, const double *__restrict__ norm, Grid g, Bag w)
{
    const double d = norm[0];
    const size_t n = (size_t)g.nx * (size_t)g.np;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        f[e] = (T)(waterbag_raw(g, w, (int)(e % (size_t)g.nx), (int)(e / (size_t)g.nx)) / d);
}

template <typename T>
__global__ void k_ic_gauss_fill(T *__restrict__ f, const double *__restrict__ e, const double *__restrict__ c,
                                const double *__restrict__ norm, Grid g)
{
    const double d = norm[0];
    const size_t n = (size_t)g.nx * (size_t)g.np;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        f[k] = (T)((e[k / (size_t)g.nx] * c[k % (size_t)g.nx]) / d);
}

// Half-widths of the HMF waterbag of magnetization M0 and energy U (Sec.
// 4.2): M0 = sin(theta0)/theta0, U = p0^2/6 + (1 - M0^2)/2.
bool hmf_halfwidths(double U, double M0, double &theta0, double &p0)
{
    if (!(M0 >= 0.0 && M0 < 1.0)) return false;
    const double kin = U - 0.5 * (1.0 - M0 * M0);
    if (!(kin >= 0.0)) return false;
    double lo = 0.0, hi = M_PI;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double val = mid > 0.0 ? sin(mid) / mid : 1.0;
        if (val > M0)
            lo = mid;
        else
            hi = mid;
        if (hi - lo <= 4e-16 * hi) break;
    }
    theta0 = 0.5 * (lo + hi);
    p0 = sqrt(6.0 * kin);
    return true;
}

}  // namespace

namespace vlasov_detail {

std::string validate_ic(const vlasov_ic *ic)
{
    if (!ic) return "NULL initial-condition spec";
    double t0, p0;
    switch (ic->kind) {
    case VLASOV_IC_WATERBAG:
        if (!std::isfinite(ic->a0) || !std::isfinite(ic->a1) || !std::isfinite(ic->amp))
            return "waterbag half-widths and noise must be finite";
        return "";
    case VLASOV_IC_WATERBAG_UM:
        if (!std::isfinite(ic->amp)) return "waterbag noise must be finite";
        if (!hmf_halfwidths(ic->a0, ic->a1, t0, p0)) return "waterbag (U, M0): need 0 <= M0 < 1 and U >= (1 - M0^2)/2";
        return "";
    case VLASOV_IC_GAUSSIAN:
        if (!(ic->a0 > 0.0) || !std::isfinite(ic->a0) || !(fabs(ic->amp) < 1.0)) return "gaussian: need T > 0 and |amp| < 1";
        return "";
    default:
        return "unknown initial-condition kind";
    }
}

}  // namespace vlasov_detail

namespace {

int launch_grid(size_t n)
{
    const size_t wg = (n + 255) / 256;
    return (int)(wg < 8192 ? (wg ? wg : 1) : 8192);
}

}  // namespace

extern "C" {

int vlasov_generate_ic(vlasov_ctx *c, const vlasov_ic *ic)
{
    if (!c || !ic) return fail(VLASOV_E_INVAL, "NULL argument");
    const vlasov_params &P = c->P;
    Grid g{(int)P.nx, (int)P.np, P.xmin, c->dx, P.pmin, c->dp};
    const size_t N = (size_t)P.nx * (size_t)P.np;
    // scratch: raw values over the whole f pair (N doubles fit in it for both
    // storages), row sums in the density partial sums (nblk nx >= np), the
    // divisor in rho; the Gaussian's node factors in the second f buffer (np
    // values) and the diagnostics columns (nx values)
    double *raw = reinterpret_cast<double *>(c->f[0]);
    double *rows = c->at<double>(c->L.part);
    double *norm = c->at<double>(c->L.rho);
    const bool f32 = P.storage == VLASOV_F32;
    void *out = c->f[0];
    const int G = launch_grid(N);
    const std::string why = validate_ic(ic);
    if (!why.empty()) return fail(VLASOV_E_INVAL, why);
    if (ic->kind == VLASOV_IC_WATERBAG || ic->kind == VLASOV_IC_WATERBAG_UM) {
        Bag w{ic->a0, ic->a1, ic->amp, ic->seed};
        if (ic->kind == VLASOV_IC_WATERBAG_UM) (void)hmf_halfwidths(ic->a0, ic->a1, w.x0, w.p0);
        w.x0 = std::max(w.x0, 2.0 * c->dx);
        w.p0 = std::max(w.p0, 2.0 * c->dp);
        k_ic_bag_raw<<<G, 256, 0, c->stream>>>(raw, g, w);
        k_ic_rows_raw<<<(g.np + 63) / 64, 64, 0, c->stream>>>(raw, rows, g);
        k_ic_norm<<<1, 64, 0, c->stream>>>(rows, norm, g);
        if (f32)
            k_ic_bag_fill<float><<<G, 256, 0, c->stream>>>((float *)out, norm, g, w);
        else
            k_ic_bag_fill<double><<<G, 256, 0, c->stream>>>((double *)out, norm, g, w);
    } else if (ic->kind == VLASOV_IC_GAUSSIAN) {
        const double T = ic->a0, A = ic->amp;
        const double phi = ic->seed == 0 ? 0.0 : 2.0 * M_PI * uniform01(ic->seed, 0);
        std::vector<double> e((size_t)P.np), cc((size_t)P.nx);
        for (int64_t j = 0; j < P.np; ++j) {
            const double v = P.pmin + (double)j * c->dp;
            e[(size_t)j] = exp(-(v * v) / (2.0 * T));
        }
        for (int64_t i = 0; i < P.nx; ++i) {
            const double x = P.xmin + (double)i * c->dx;
            cc[(size_t)i] = 1.0 + A * cos(x - phi);
        }
        double *de = reinterpret_cast<double *>(c->f[1]);
        double *dc = c->at<double>(c->L.mom_col);
        HIP_TRY(hipMemcpyAsync(de, e.data(), e.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(dc, cc.data(), cc.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        k_ic_rows_gauss<<<(g.np + 63) / 64, 64, 0, c->stream>>>(de, dc, rows, g);
        k_ic_norm<<<1, 64, 0, c->stream>>>(rows, norm, g);
        if (f32)
            k_ic_gauss_fill<float><<<G, 256, 0, c->stream>>>((float *)out, de, dc, norm, g);
        else
            k_ic_gauss_fill<double><<<G, 256, 0, c->stream>>>((double *)out, de, dc, norm, g);
    }
    int rc = check_launch("initial condition");
    if (rc != VLASOV_OK) return rc;
    double d = 0.0;
    HIP_TRY(hipMemcpyAsync(&d, norm, sizeof d, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));  // also keeps the host tables alive until copied
    if (!(d > 0.0) || !std::isfinite(d)) return fail(VLASOV_E_INVAL, "the initial condition has no mass on the grid");
    c->cur = 0;
    return VLASOV_OK;
}

}  // extern "C"
