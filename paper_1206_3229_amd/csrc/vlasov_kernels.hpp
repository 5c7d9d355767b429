// Device kernels of the split semi-Lagrangian Vlasov step for gfx950.
//
// Arithmetic contract (shared by every kernel here, compiled with
// -ffp-contract=off): products and sums round where written, fused
// multiply-adds appear only as explicit fma()/fmaf().  Every sum over an index
// of length n uses 64 interleaved running sums (term t in partial t mod 64,
// ascending t; the 64 lanes of a wavefront) combined by the xor butterfly
// d = 32, 16, ..., 1, so results do not depend on launch shapes.  Column sums
// over the momentum rows are serial inside blocks of 16 consecutive rows and
// then use that 64-way rule over the block index.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace vk {

enum { BC_PERIODIC = 0, BC_ZERO = 1 };
constexpr int ROWS_PER_BLOCK = 16;  // rows of one density partial sum

// ---------------------------------------------------------------------------
// Eq. (findif): eighth-order centred second difference (without 1/du^2; the
// du^2 of the spline coefficients of eq. (splinecoeffs) cancels it).
// ---------------------------------------------------------------------------
template <typename T> struct FD;
template <> struct FD<double> {
    static constexpr double c0 = -205.0 / 72.0, c1 = 8.0 / 5.0, c2 = -1.0 / 5.0, c3 = 8.0 / 315.0,
                            c4 = -1.0 / 560.0;
};
template <> struct FD<float> {
    static constexpr float c0 = (float)(-205.0 / 72.0), c1 = (float)(8.0 / 5.0), c2 = (float)(-1.0 / 5.0),
                           c3 = (float)(8.0 / 315.0), c4 = (float)(-1.0 / 560.0);
};

__device__ __forceinline__ double vfma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float vfma(float a, float b, float c) { return fmaf(a, b, c); }

// x points at the centre sample; reads x[-4..4].  Symmetric pairs first,
// accumulated from the outermost pair inwards.
template <typename T>
__device__ __forceinline__ T second_diff(const T *x)
{
    T s = FD<T>::c4 * (x[-4] + x[4]);
    s = vfma(FD<T>::c3, x[-3] + x[3], s);
    s = vfma(FD<T>::c2, x[-2] + x[2], s);
    s = vfma(FD<T>::c1, x[-1] + x[1], s);
    return vfma(FD<T>::c0, x[0], s);
}

// Eq. (splinegen) on the cell [k, k+1]: alpha f_k + beta f_k+1 + gamma D_k +
// delta D_k+1, accumulated in the order gamma, delta, beta, alpha.
template <typename T>
__device__ __forceinline__ T spline(T a, T b, T g, T d, T fk, T fk1, T Dk, T Dk1)
{
    T r = g * Dk;
    r = vfma(d, Dk1, r);
    r = vfma(b, fk1, r);
    return vfma(a, fk, r);
}

// ---------------------------------------------------------------------------
// Foot of the characteristic (Sec. 3): the new value at node i is the spline
// at i + xi cells, xi = -shift.  m = floor(xi), theta = xi - m (a rounded
// theta of 1 becomes 0 with m + 1); alpha = 1 - theta, beta = theta,
// gamma = (alpha^3 - alpha)/6, delta = (beta^3 - beta)/6.  A non-finite or
// huge shift gives m = 0 and NaN weights.
// ---------------------------------------------------------------------------
struct Foot {
    int64_t m;
    double a, b, g, d;
};

__host__ __device__ inline Foot foot_of_shift(double shift)
{
    Foot w;
    double xi = -shift;
    if (!(fabs(xi) < 2147483648.0)) {
        w.m = 0;
        w.a = w.b = w.g = w.d = __builtin_nan("");
        return w;
    }
    double fl = floor(xi);
    double th = xi - fl;
    w.m = (int64_t)fl;
    if (th >= 1.0) {
        th = 0.0;
        w.m += 1;
    }
    w.a = 1.0 - th;
    w.b = th;
    w.g = ((w.a * w.a) * w.a - w.a) / 6.0;
    w.d = ((w.b * w.b) * w.b - w.b) / 6.0;
    return w;
}

// Foot offset as used by the kernels: reduced to [0, n) on a periodic axis;
// clamped to +-(n + 16) with zero extension (beyond that every sample is 0).
__host__ __device__ inline int32_t reduce_offset(int64_t m, int64_t n, int bc)
{
    if (bc == BC_PERIODIC) {
        int64_t r = m % n;
        if (r < 0) r += n;
        return (int32_t)r;
    }
    int64_t lim = n + 16;
    return (int32_t)(m > lim ? lim : (m < -lim ? -lim : m));
}

__device__ __forceinline__ int wrap(int q, int n)
{
    int r = q % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = v + __shfl_xor(v, d, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Steps 1 and 4 (eqs. step1, step4): drift along x, row j shifted by the
// constant p_j tau/dx cells.  NPASS = 2 applies the half drift twice (the
// second half drift of one step and the first of the next), keeping the
// intermediate row in LDS.  One workgroup: TW consecutive columns of 16
// consecutive rows; the input window of each row is staged in LDS with its
// halo (periodic wrap or zeros).  With PARTIALS, also writes the serial
// column sum of the 16 output rows (density partial sums).
// ---------------------------------------------------------------------------
template <typename T, int NPASS, int BC, bool PARTIALS, int TW>
__global__ __launch_bounds__(TW) void k_drift(const T *__restrict__ fin, T *__restrict__ fout,
                                              const int32_t *__restrict__ dm, const double4 *__restrict__ dw,
                                              double *__restrict__ part, int nx, int np)
{
    constexpr int WIN = TW + 9 * NPASS;
    __shared__ T win[WIN];
    __shared__ T mid[NPASS == 2 ? TW + 9 : 1];
    const int t = threadIdx.x;
    const int i0 = blockIdx.x * TW;
    const int i = i0 + t;
    const int j0 = blockIdx.y * ROWS_PER_BLOCK;
    const int jend = min(j0 + ROWS_PER_BLOCK, np);
    double acc = 0.0;
    for (int j = j0; j < jend; ++j) {
        const int m = dm[j];
        const double4 w = dw[j];
        const T a = (T)w.x, b = (T)w.y, g = (T)w.z, d = (T)w.w;
        const T *row = fin + (size_t)j * nx;
        // win[s] holds the sample at global position base + s
        const int base = i0 + NPASS * m - 4 * NPASS;
        for (int s = t; s < WIN; s += TW) {
            const int q = base + s;
            T v;
            if (BC == BC_PERIODIC)
                v = row[wrap(q, nx)];
            else
                v = (q >= 0 && q < nx) ? row[q] : T(0);
            win[s] = v;
        }
        __syncthreads();
        const T *src = win;
        if (NPASS == 2) {
            // first half drift at positions i0 + m - 4 + u, u in [0, TW + 9)
            for (int u = t; u < TW + 9; u += TW) {
                const T *x = win + u + 4;
                T v = spline(a, b, g, d, x[0], x[1], second_diff(x), second_diff(x + 1));
                if (BC == BC_ZERO) {
                    const int q = i0 + m - 4 + u;
                    if (q < 0 || q >= nx) v = T(0);
                }
                mid[u] = v;
            }
            __syncthreads();
            src = mid;
        }
        const T *x = src + t + 4;
        const T v = spline(a, b, g, d, x[0], x[1], second_diff(x), second_diff(x + 1));
        if (i < nx) {
            fout[(size_t)j * nx + i] = v;
            if (PARTIALS) acc = acc + (double)v;
        }
        __syncthreads();
    }
    if (PARTIALS && i < nx) part[(size_t)blockIdx.y * nx + i] = acc;
}

// ---------------------------------------------------------------------------
// Step 3 (eq. step3): kick along p, column i shifted by F_i dt/dp cells.  One
// thread per column and R consecutive output rows; the R + 9 samples of the
// column window are held in registers (lanes of a wavefront read adjacent
// columns of the same rows).
// ---------------------------------------------------------------------------
template <typename T, int BC, int R>
__global__ __launch_bounds__(256) void k_kick(const T *__restrict__ fin, T *__restrict__ fout,
                                              const double *__restrict__ F, double dt, double dp, int nx, int np)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    const int j0 = blockIdx.y * R;
    const Foot ft = foot_of_shift((F[i] * dt) / dp);
    const int m = reduce_offset(ft.m, np, BC);
    const T a = (T)ft.a, b = (T)ft.b, g = (T)ft.g, d = (T)ft.d;
    const int base = j0 + m - 4;
    T w[R + 10];
#pragma unroll
    for (int s = 0; s < R + 10; ++s) {
        const int q = base + s;
        if (BC == BC_PERIODIC)
            w[s] = fin[(size_t)wrap(q, np) * nx + i];
        else
            w[s] = (q >= 0 && q < np) ? fin[(size_t)q * nx + i] : T(0);
    }
    T D[R + 1];
#pragma unroll
    for (int r = 0; r <= R; ++r) D[r] = second_diff(w + r + 4);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        if (j < np) fout[(size_t)j * nx + i] = spline(a, b, g, d, w[r + 4], w[r + 5], D[r], D[r + 1]);
    }
}

// ---------------------------------------------------------------------------
// Density rho_i = dp * sum_j f_ji from the 16-row partial sums: one wavefront
// per column, lane l sums the blocks b = l mod 64 in ascending order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_density(const double *__restrict__ part, double *__restrict__ rho, int nx,
                                                 int nblk, double dp)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nx) return;
    double acc = 0.0;
    for (int b = lane; b < nblk; b += 64) acc = acc + part[(size_t)b * nx + i];
    acc = wave_sum(acc);
    if (lane == 0) rho[i] = dp * acc;
}

// Magnetization of eq. (mxmydef) by one wavefront; lane 0 returns (mx, my).
__device__ inline void magnetization(const double *__restrict__ rho, const double *__restrict__ cs,
                                     const double *__restrict__ sn, int n, double dx, double &mx, double &my)
{
    const int lane = threadIdx.x & 63;
    double c = 0.0, s = 0.0;
    for (int i = lane; i < n; i += 64) {
        c = fma(cs[i], rho[i], c);
        s = fma(sn[i], rho[i], s);
    }
    c = wave_sum(c);
    s = wave_sum(s);
    mx = dx * c;
    my = dx * s;
}

// Keeps (mx, my) of the latest force evaluation and appends it to the history.
__device__ inline void record_history(double *mxmy, double *hist, int64_t *hcount, int64_t hcap, double mx,
                                      double my)
{
    mxmy[0] = mx;
    mxmy[1] = my;
    if (hcap <= 0) return;
    const int64_t c = *hcount;
    if (c < hcap) {
        hist[2 * c] = mx;
        hist[2 * c + 1] = my;
    }
    *hcount = c + 1;
}

// HMF force, eq. (hmfmeanforce): F_i = -sin(x_i) M_x + cos(x_i) M_y.  One
// workgroup; wavefront 0 forms (M_x, M_y).
__global__ __launch_bounds__(256) void k_force_hmf(const double *__restrict__ rho, const double *__restrict__ cs,
                                                   const double *__restrict__ sn, double *__restrict__ F, int n,
                                                   double dx, double *mxmy, double *hist, int64_t *hcount,
                                                   int64_t hcap)
{
    __shared__ double M[2];
    if (threadIdx.x < 64) {
        double mx, my;
        magnetization(rho, cs, sn, n, dx, mx, my);
        if (threadIdx.x == 0) {
            M[0] = mx;
            M[1] = my;
            record_history(mxmy, hist, hcount, hcap, mx, my);
        }
    }
    __syncthreads();
    const double mx = M[0], my = M[1];
    for (int i = threadIdx.x; i < n; i += blockDim.x) F[i] = fma(my, cs[i], -(mx * sn[i]));
}

// Magnetization only (ring model).  One wavefront.
__global__ __launch_bounds__(64) void k_magnetization(const double *__restrict__ rho, const double *__restrict__ cs,
                                                      const double *__restrict__ sn, int n, double dx, double *mxmy,
                                                      double *hist, int64_t *hcount, int64_t hcap)
{
    double mx, my;
    magnetization(rho, cs, sn, n, dx, mx, my);
    if (threadIdx.x == 0) record_history(mxmy, hist, hcount, hcap, mx, my);
}

// Ring force, eq. (meanforce) with eq. (ringpot): F_i = -dx sum_k K_{(i-k)
// mod n} rho_k with K the tabulated V'.  One wavefront per output.
__global__ __launch_bounds__(256) void k_force_ring(const double *__restrict__ rho, const double *__restrict__ K,
                                                    double *__restrict__ F, int n, double dx)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    double acc = 0.0;
    for (int k = lane; k < n; k += 64) {
        int d = i - k;
        if (d < 0) d += n;
        acc = fma(K[d], rho[k], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) F[i] = -(dx * acc);
}

// Sheet force, eq. (sheetpot) with V = 2 pi G |x|: F_i = K (S - 2 P_i - rho_i),
// K = 2 pi G dx, P_i the exclusive prefix sum of rho and S its total.  One
// wavefront: lane l scans the contiguous chunk [l c, (l+1) c), c = ceil(n/64);
// chunk totals by an inclusive Hillis-Steele scan d = 1, 2, ..., 32.
__global__ __launch_bounds__(64) void k_force_sheet(const double *__restrict__ rho, double *__restrict__ F, int n,
                                                    double K)
{
    const int l = threadIdx.x;
    const int c = (n + 63) / 64;
    const int lo = l * c;
    const int hi = min(lo + c, n);
    double tot = 0.0;
    for (int i = lo; i < hi; ++i) tot = tot + rho[i];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double v = __shfl_up(tot, d, 64);
        if (l >= d) tot = v + tot;
    }
    double excl = __shfl_up(tot, 1, 64);
    if (l == 0) excl = 0.0;
    const double S = __shfl(tot, 63, 64);
    double acc = 0.0;
    for (int i = lo; i < hi; ++i) {
        const double Pi = excl + acc;
        F[i] = K * (fma(-2.0, Pi, S) - rho[i]);
        acc = acc + rho[i];
    }
}

// ---------------------------------------------------------------------------
// Diagnostics.  Pass 1: 16-row block sums of f, p f, p^2/2 f and f^2.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_mom_blocks(const T *__restrict__ f, double *__restrict__ scratch, int nx,
                                                    int np, int nblk, double pmin, double dp)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    const int b = blockIdx.y;
    const int j0 = b * ROWS_PER_BLOCK;
    const int jend = min(j0 + ROWS_PER_BLOCK, np);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = j0; j < jend; ++j) {
        const double v = (double)f[(size_t)j * nx + i];
        const double pj = pmin + (double)j * dp;
        const double kj = 0.5 * (pj * pj);
        s0 = s0 + v;
        s1 = fma(pj, v, s1);
        s2 = fma(kj, v, s2);
        s3 = fma(v, v, s3);
    }
    const size_t plane = (size_t)nblk * nx;
    const size_t o = (size_t)b * nx + i;
    scratch[o] = s0;
    scratch[plane + o] = s1;
    scratch[2 * plane + o] = s2;
    scratch[3 * plane + o] = s3;
}

// Pass 2: column quantities col[q][i] = dp * sum over blocks (one wavefront
// per column).
__global__ __launch_bounds__(256) void k_mom_cols(const double *__restrict__ scratch, double *__restrict__ col,
                                                  int nx, int nblk, double dp)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nx) return;
    const size_t plane = (size_t)nblk * nx;
    for (int q = 0; q < 4; ++q) {
        double acc = 0.0;
        for (int b = lane; b < nblk; b += 64) acc = acc + scratch[q * plane + (size_t)b * nx + i];
        acc = wave_sum(acc);
        if (lane == 0) col[(size_t)q * nx + i] = dp * acc;
    }
}

// Pass 3 (ring and sheet): phi_i = sum_k V(x_i - x_k) rho_k with V the
// tabulated ring potential, or |i - k| (sheet, in cells).
template <bool RING>
__global__ __launch_bounds__(256) void k_mom_phi(const double *__restrict__ rho, const double *__restrict__ V,
                                                 double *__restrict__ phi, int n)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    double acc = 0.0;
    for (int k = lane; k < n; k += 64) {
        double v;
        if (RING) {
            int d = i - k;
            if (d < 0) d += n;
            v = V[d];
        } else {
            v = (double)(i > k ? i - k : k - i);
        }
        acc = fma(v, rho[k], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) phi[i] = acc;
}

// Pass 4: totals (one wavefront).  out = {mass, momentum, kinetic, potential,
// energy, mx, my, l2}.
__global__ __launch_bounds__(64) void k_mom_final(const double *__restrict__ col, const double *__restrict__ phi,
                                                  const double *__restrict__ cs, const double *__restrict__ sn,
                                                  double *__restrict__ out, int n, double dx, int model,
                                                  double wcoef)
{
    const int lane = threadIdx.x;
    const double *rho = col, *jj = col + n, *kk = col + 2 * n, *qq = col + 3 * n;
    double sm = 0.0, sj = 0.0, sk = 0.0, sq = 0.0, c = 0.0, s = 0.0, w = 0.0;
    const bool angular = (model == 0 || model == 1);
    const bool pair = (model == 1 || model == 2);
    for (int i = lane; i < n; i += 64) {
        sm = sm + rho[i];
        sj = sj + jj[i];
        sk = sk + kk[i];
        sq = sq + qq[i];
        if (angular) {
            c = fma(cs[i], rho[i], c);
            s = fma(sn[i], rho[i], s);
        }
        if (pair) w = fma(phi[i], rho[i], w);
    }
    sm = wave_sum(sm);
    sj = wave_sum(sj);
    sk = wave_sum(sk);
    sq = wave_sum(sq);
    c = wave_sum(c);
    s = wave_sum(s);
    w = wave_sum(w);
    if (lane == 0) {
        const double mass = dx * sm, kin = dx * sk;
        double mx = 0.0, my = 0.0, W = 0.0;
        if (angular) {
            mx = dx * c;
            my = dx * s;
        }
        if (model == 0)
            W = 0.5 * ((mass * mass - mx * mx) - my * my);
        else if (pair)
            W = wcoef * w;
        out[0] = mass;
        out[1] = dx * sj;
        out[2] = kin;
        out[3] = W;
        out[4] = kin + W;
        out[5] = mx;
        out[6] = my;
        out[7] = dx * sq;
    }
}

// Streaming copy (bandwidth ceiling): 16-byte vectors, grid-stride.
__global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) dst[k] = src[k];
}

}  // namespace vk
