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

// Marks loaded values as used here, after all of their loads, so that the
// compiler issues the loads together before any branch that follows (a load
// whose only use is conditional is otherwise moved into the branch, next to
// a wait for it).
template <typename T> __device__ __forceinline__ void keep_issued(T &v) { __asm__ __volatile__("" : "+v"(v)); }

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

// One sample of a line of n values (stride between samples `stride`) under
// the boundary rule of the axis.
template <typename T, int BC>
__device__ __forceinline__ T sample(const T *__restrict__ line, int q, int n, size_t stride)
{
    if (BC == BC_PERIODIC) return line[(size_t)wrap(q, n) * stride];
    return (q >= 0 && q < n) ? line[(size_t)q * stride] : T(0);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = v + __shfl_xor(v, d, 64);
    return v;
}

// Tile placement.  Workgroups are dispatched to the 8 XCDs of the chip in
// round-robin order of their linear id; each XCD is given a contiguous band of
// tile rows (x fastest inside the band) so that tiles sharing halo lines are
// served by the same L2.  Launch 8 * ceil(nty/8) * ntx workgroups.
constexpr int NXCD = 8;

__host__ __device__ inline int xcd_grid(int ntx, int nty) { return NXCD * ((nty + NXCD - 1) / NXCD) * ntx; }

__device__ __forceinline__ bool xcd_tile(int ntx, int nty, int &tx, int &ty)
{
    const int id = blockIdx.x;
    const int k = id / NXCD;
    const int per = (nty + NXCD - 1) / NXCD;
    ty = (id % NXCD) * per + k / ntx;
    tx = k % ntx;
    return ty < nty;
}

// Two adjacent values as one 8- or 16-byte vector.
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
template <typename T> struct Vec4;
template <> struct Vec4<double> { using type = double4; };
template <> struct Vec4<float> { using type = float4; };

// Interpolates the V adjacent outputs q = V u .. V u + V - 1 of a row from an
// LDS window `src` (the sample at the start of output q's cell is src[q + 4]):
// V + 1 stencils shared by the run, read as V/2 + 5 aligned pairs
// src[V u .. V u + V + 9].
template <typename T, int V>
__device__ __forceinline__ void spline_run(const T *src, int u, T a, T b, T g, T d, T (&o)[V])
{
    using V2 = typename Vec2<T>::type;
    static_assert(V % 2 == 0, "runs of even length");
    const V2 *p = reinterpret_cast<const V2 *>(src) + (V / 2) * u;
    T x[V + 10];
#pragma unroll
    for (int k = 0; k < V / 2 + 5; ++k) {
        const V2 v = p[k];
        x[2 * k] = v.x;
        x[2 * k + 1] = v.y;
    }
    T D[V + 1];
#pragma unroll
    for (int k = 0; k <= V; ++k) D[k] = second_diff(x + 4 + k);
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = spline(a, b, g, d, x[4 + k], x[5 + k], D[k], D[k + 1]);
}

// Stores V adjacent outputs at row[i .. i + V), vectorised when aligned.
template <typename T, int V>
__device__ __forceinline__ void store_run(T *row, int i, int nx, const T (&o)[V])
{
    using V2 = typename Vec2<T>::type;
    if (i + V <= nx && (nx & 1) == 0) {
#pragma unroll
        for (int k = 0; k < V; k += 2) {
            V2 w;
            w.x = o[k];
            w.y = o[k + 1];
            *reinterpret_cast<V2 *>(row + i + k) = w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k)
            if (i + k < nx) row[i + k] = o[k];
    }
}

// ---------------------------------------------------------------------------
// Steps 1 and 4 (eqs. step1, step4): drift along x, row j shifted by the
// constant p_j tau/dx cells.  NPASS = 2 applies two half drifts in turn (the
// second half drift of one (sub)step and the first of the next, tables 1 and
// 2: equal for the Strang splitting), keeping the intermediate row in LDS.
// One workgroup of NT threads: TW consecutive columns of a block of 16
// consecutive rows, runs of V adjacent columns per thread; TW = V NT - TRIM
// (a trim keeps the TW + 9 intermediate values of the two-pass form within
// one run per thread).  Rows stream through two LDS window
// buffers; the window of each row (TW columns plus the stencil and shift halo,
// periodic wrap or zeros) is requested PF rows ahead of its use and held in
// registers meanwhile.  With PARTIALS, also writes the serial column sum of the
// 16 output rows (density partial sums).
// ---------------------------------------------------------------------------
template <typename T, int BC, int NPASS, int TW, int NT, int NLD>
__device__ __forceinline__ void load_window(const T *__restrict__ fin, const int32_t *__restrict__ dm1,
                                            const int32_t *__restrict__ dm2, int j, int i0, int nx, T (&v)[NLD],
                                            uint32_t &inside)
{
    // Branch-free: every thread issues NLD loads at valid addresses (periodic
    // positions wrapped, zero-extended ones clamped; slots past the window
    // load a duplicate that is never used). For zero extension bit k of
    // `inside` says whether slot k lies in the grid; the zero is applied when
    // the value is written to LDS, not here, so that no use of a loaded value
    // sits next to its load and the loads of the rows requested ahead stay in
    // flight.
    const T *row = fin + (size_t)j * nx;
    int base = i0 + (NPASS == 2 ? dm1[j] + dm2[j] : dm1[j]) - 4 * NPASS;
    if (BC == BC_PERIODIC) base = wrap(base, nx);
    inside = 0;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int s = threadIdx.x + k * NT;
        int q = base + s;
        if (BC == BC_PERIODIC) {
            q = q >= nx ? q - nx : q;
            q = q >= nx ? wrap(q, nx) : q;
            v[k] = row[q];
        } else {
            v[k] = row[min(max(q, 0), nx - 1)];
            inside |= (uint32_t)(q >= 0 && q < nx) << k;
        }
    }
}

// Geometry of a drift tile: NT threads, runs of V columns, TW = V NT - TRIM
// columns; buffer sizes of the row window and of the first-pass row.
template <int NPASS, int NT, int V, int TRIM>
struct DriftGeom {
    static constexpr int TW = V * NT - TRIM;
    static constexpr int WIN = TW + 9 * NPASS;        // window samples per row
    static constexpr int MIDN = TW + 9;               // first-pass outputs per row (NPASS = 2)
    static constexpr int NRUN1 = (MIDN + V - 1) / V;  // first-pass runs per row
    static constexpr int NLD = (WIN + NT - 1) / NT;   // loads per thread per row
    // runs read V + 10 samples from V u: pad the buffers past the last run
    static constexpr int LDW = ((NPASS == 2 ? NRUN1 * V : TW) + 10 + 1) & ~1;
    static constexpr int MIDW = NRUN1 * V > TW + 10 ? NRUN1 * V : TW + 10;
    static constexpr int LDM = NPASS == 2 ? (MIDW + 1) & ~1 : 2;
    // allocation pitch of a window buffer: slot LDW takes the writes of lanes
    // past the window, so that the LDS write (the only use of a prefetched
    // value) is unconditional and the compiler cannot sink the load into a
    // branch next to it
    static constexpr int LDA = LDW + 2;
    static_assert(TRIM % V == 0 && TW > 0, "tile width a positive multiple of the run");
    static_assert(LDW >= WIN, "window buffer");
};

template <int NT, int V, int TRIM>
struct DriftShape {
    static constexpr int TW = V * NT - TRIM;
};

// One drift tile (columns [tx TW, (tx+1) TW) of rows [16 ty, 16 ty + 16)).
// win: two LDS row buffers of at least LDA entries each, mid: LDS row of LDM
// (NPASS = 2).
// FULL: the tile has all 16 rows and all TW columns inside the grid and nx is
// even; then the row loop is straight-line code (no branch around a memory
// access), which lets the loads requested ahead stay in flight.
template <typename T, int NPASS, int BC, bool PARTIALS, int NT, int V, int TRIM, int PF, bool FULL>
__device__ __forceinline__ void drift_tile(const T *__restrict__ fin, T *__restrict__ fout,
                                           const int32_t *__restrict__ dm1, const double4 *__restrict__ dw1,
                                           const int32_t *__restrict__ dm2, const double4 *__restrict__ dw2,
                                           double *__restrict__ part, int nx, int np, int tx, int ty, T *win0,
                                           T *win1, T *mid)
{
    using G = DriftGeom<NPASS, NT, V, TRIM>;
    constexpr int R = ROWS_PER_BLOCK;
    constexpr int TW = G::TW, WIN = G::WIN, MIDN = G::MIDN, NRUN1 = G::NRUN1, NLD = G::NLD, LDW = G::LDW,
                  LDM = G::LDM;
    const int t = threadIdx.x;
    const int i0 = tx * TW;
    const int j0 = ty * R;
    const int nr = FULL ? R : min(R, np - j0);

    for (int s = WIN + t; s < LDW; s += NT) {
        win0[s] = T(0);
        win1[s] = T(0);
    }
    if (NPASS == 2)
        for (int s = MIDN + t; s < LDM; s += NT) mid[s] = T(0);

    T v[PF][NLD];
    uint32_t inside[PF];
    static_assert(NLD <= 32, "one bit per loaded slot");
#pragma unroll
    for (int r = 0; r < PF; ++r)
        if (FULL || r < nr) load_window<T, BC, NPASS, TW, NT, NLD>(fin, dm1, dm2, j0 + r, i0, nx, v[r], inside[r]);

    const int i = i0 + V * t;                // first of this thread's V columns
    const bool own = FULL || V * t < TW;     // trailing threads own no output when TRIM > 0
    double acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (FULL || r < nr) {
            T *wrow = (r & 1) ? win1 : win0;
#pragma unroll
            for (int k = 0; k < NLD; ++k) {
                // slots k < NLD - 1 always lie in the window (t < NT)
                const int s = t + k * NT;
                const T x = v[r % PF][k];
                wrow[k < NLD - 1 || s < WIN ? s : LDW] = BC == BC_PERIODIC || (inside[r % PF] >> k & 1u) ? x : T(0);
            }
            if (FULL ? r + PF < R : r + PF < nr)
                load_window<T, BC, NPASS, TW, NT, NLD>(fin, dm1, dm2, j0 + r + PF, i0, nx, v[r % PF],
                                                       inside[r % PF]);
            __syncthreads();
            const int j = j0 + r;
            const double4 w = (NPASS == 2 ? dw2 : dw1)[j];
            const T a = (T)w.x, b = (T)w.y, g = (T)w.z, d = (T)w.w;
            const T *src = wrow;
            if (NPASS == 2) {
                // first half drift (table 1) at the positions i0 + m - 4 + q,
                // q in [0, TW + 9), that the second (table 2, offset m) reads
                const int m = dm2[j];
                const double4 w1 = dw1[j];
                const T a1 = (T)w1.x, b1 = (T)w1.y, g1 = (T)w1.z, d1 = (T)w1.w;
                for (int u = t; u < NRUN1; u += NT) {
                    T o[V];
                    spline_run<T, V>(src, u, a1, b1, g1, d1, o);
                    if (BC == BC_ZERO) {
                        const int q = i0 + m - 4 + V * u;
#pragma unroll
                        for (int k = 0; k < V; ++k)
                            if (q + k < 0 || q + k >= nx) o[k] = T(0);
                    }
#pragma unroll
                    for (int k = 0; k < V; k += 2) {
                        typename Vec2<T>::type ww;
                        ww.x = o[k];
                        ww.y = o[k + 1];
                        reinterpret_cast<typename Vec2<T>::type *>(mid + V * u)[k / 2] = ww;
                    }
                }
                __syncthreads();
                src = mid;
            }
            if (own) {
                T o[V];
                spline_run<T, V>(src, t, a, b, g, d, o);
                if (FULL) {
#pragma unroll
                    for (int k = 0; k < V; k += 2) {
                        typename Vec2<T>::type ww;
                        ww.x = o[k];
                        ww.y = o[k + 1];
                        *reinterpret_cast<typename Vec2<T>::type *>(fout + (size_t)j * nx + i + k) = ww;
                    }
                } else {
                    store_run<T, V>(fout + (size_t)j * nx, i, nx, o);
                }
                if (PARTIALS) {
#pragma unroll
                    for (int k = 0; k < V; ++k) acc[k] = acc[k] + (double)o[k];
                }
            }
        }
    }
    if (PARTIALS && own) {
        double *prow = part + (size_t)ty * nx;
#pragma unroll
        for (int k = 0; k < V; ++k)
            if (FULL || i + k < nx) prow[i + k] = acc[k];
    }
}

// Full tiles take the straight-line form, edge tiles the guarded one.
template <typename T, int NPASS, int BC, bool PARTIALS, int NT, int V, int TRIM, int PF>
__device__ __forceinline__ void drift_tile_any(const T *__restrict__ fin, T *__restrict__ fout,
                                               const int32_t *__restrict__ dm1, const double4 *__restrict__ dw1,
                                               const int32_t *__restrict__ dm2, const double4 *__restrict__ dw2,
                                               double *__restrict__ part, int nx, int np, int tx, int ty, T *win0,
                                               T *win1, T *mid)
{
    constexpr int TW = DriftGeom<NPASS, NT, V, TRIM>::TW;
    const bool full = (ty + 1) * ROWS_PER_BLOCK <= np && (tx + 1) * TW <= nx && (nx & 1) == 0;
    if (full)
        drift_tile<T, NPASS, BC, PARTIALS, NT, V, TRIM, PF, true>(fin, fout, dm1, dw1, dm2, dw2, part, nx, np, tx, ty,
                                                                  win0, win1, mid);
    else
        drift_tile<T, NPASS, BC, PARTIALS, NT, V, TRIM, PF, false>(fin, fout, dm1, dw1, dm2, dw2, part, nx, np, tx, ty,
                                                                   win0, win1, mid);
}

template <typename T, int NPASS, int BC, bool PARTIALS, int NT, int V, int TRIM, int PF>
static __global__ __launch_bounds__(NT) void k_drift(const T *__restrict__ fin, T *__restrict__ fout,
                                              const int32_t *__restrict__ dm1, const double4 *__restrict__ dw1,
                                              const int32_t *__restrict__ dm2, const double4 *__restrict__ dw2,
                                              double *__restrict__ part, int nx, int np, int ntx, int nty)
{
    using G = DriftGeom<NPASS, NT, V, TRIM>;
    __shared__ __attribute__((aligned(16))) T win[2][G::LDA];
    __shared__ __attribute__((aligned(16))) T mid[G::LDM];
    int tx, ty;
    if (!xcd_tile(ntx, nty, tx, ty)) return;
    drift_tile_any<T, NPASS, BC, PARTIALS, NT, V, TRIM, PF>(fin, fout, dm1, dw1, dm2, dw2, part, nx, np, tx, ty, win[0],
                                                            win[1], mid);
}

// ---------------------------------------------------------------------------
// Step 3 (eq. step3): kick along p, column i shifted by F_i dt/dp cells.  One
// thread per column and R consecutive output rows; the R + 9 samples of the
// column window are requested at once and held in registers (the lanes of a
// wavefront read adjacent columns of the same rows).
// ---------------------------------------------------------------------------
template <typename T, int BC, int R>
__device__ __forceinline__ void kick_tile(const T *__restrict__ fin, T *__restrict__ fout,
                                          const double *__restrict__ F, double dt, double dp, int nx, int np, int tx,
                                          int ty)
{
    const int i = tx * 256 + threadIdx.x;
    if (i >= nx) return;
    const int j0 = ty * R;
    const Foot ft = foot_of_shift((F[i] * dt) / dp);
    const int m = reduce_offset(ft.m, np, BC);
    const T a = (T)ft.a, b = (T)ft.b, g = (T)ft.g, d = (T)ft.d;
    const int base = j0 + m - 4;
    const T *col = fin + i;
    T w[R + 10];
#pragma unroll
    for (int s = 0; s < R + 10; ++s) w[s] = sample<T, BC>(col, base + s, np, (size_t)nx);
    T Dk = second_diff(w + 4);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T Dk1 = second_diff(w + r + 5);
        const int j = j0 + r;
        if (j < np) fout[(size_t)j * nx + i] = spline(a, b, g, d, w[r + 4], w[r + 5], Dk, Dk1);
        Dk = Dk1;
    }
}

template <typename T, int BC, int R>
static __global__ __launch_bounds__(256) void k_kick(const T *__restrict__ fin, T *__restrict__ fout,
                                              const double *__restrict__ F, double dt, double dp, int nx, int np,
                                              int ntx, int nty)
{
    int tx, ty;
    if (!xcd_tile(ntx, nty, tx, ty)) return;
    kick_tile<T, BC, R>(fin, fout, F, dt, dp, nx, np, tx, ty);
}

// ---------------------------------------------------------------------------
// The filter along p, after the last kick of a filtered step (the filtering
// the conclusions name as an extension): out_j = f_j - c s_j with c =
// sigma/256 and s_j = sum_m b_m f_{j+m}, b the binomial weights (1, -8, 28,
// -56, 70, ...) of the eighth central difference, symmetric pairs added
// first and accumulated from the outermost pair inwards.  One thread per
// column and R consecutive rows, the R + 8 samples held in registers.
// ---------------------------------------------------------------------------
template <typename T, int BC, int R>
static __global__ __launch_bounds__(256) void k_filter_p(const T *__restrict__ fin, T *__restrict__ fout, double c,
                                                  int nx, int np, int ntx, int nty)
{
    int tx, ty;
    if (!xcd_tile(ntx, nty, tx, ty)) return;
    const int i = tx * 256 + threadIdx.x;
    if (i >= nx) return;
    const int j0 = ty * R;
    const T *col = fin + i;
    T w[R + 8];
#pragma unroll
    for (int s = 0; s < R + 8; ++s) w[s] = sample<T, BC>(col, j0 - 4 + s, np, (size_t)nx);
    const T cc = (T)c;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        const T *q = w + r + 4;
        T sm = q[-4] + q[4];
        sm = vfma(T(-8), q[-3] + q[3], sm);
        sm = vfma(T(28), q[-2] + q[2], sm);
        sm = vfma(T(-56), q[-1] + q[1], sm);
        sm = vfma(T(70), q[0], sm);
        if (j < np) fout[(size_t)j * nx + i] = vfma(-cc, sm, q[0]);
    }
}

// The kick of a filtered step followed by the filter, in one pass: each
// thread kicks rows j0 - 4 .. j0 + R + 3 of its column (the filter's window;
// rows outside the grid are zero with zero extension, wrapped otherwise)
// from R + 18 samples held in registers, then filters rows j0 .. j0 + R - 1.
// Every value is computed as by k_kick and k_filter_p, so the result is the
// same bit for bit.
// ---------------------------------------------------------------------------
template <typename T, int BC, int R>
static __global__ __launch_bounds__(256) void k_kick_filter(const T *__restrict__ fin, T *__restrict__ fout,
                                                     const double *__restrict__ F, double dt, double dp, double c,
                                                     int nx, int np, int ntx, int nty)
{
    int tx, ty;
    if (!xcd_tile(ntx, nty, tx, ty)) return;
    const int i = tx * 256 + threadIdx.x;
    if (i >= nx) return;
    const int j0 = ty * R;
    const Foot ft = foot_of_shift((F[i] * dt) / dp);
    const int m = reduce_offset(ft.m, np, BC);
    const T a = (T)ft.a, b = (T)ft.b, g = (T)ft.g, d = (T)ft.d;
    const int base = j0 - 8 + m;  // sample 0: row j0 - 4 + m - 4
    const T *col = fin + i;
    T w[R + 18];
#pragma unroll
    for (int s = 0; s < R + 18; ++s) w[s] = sample<T, BC>(col, base + s, np, (size_t)nx);
    // kicked rows j0 - 4 + u, u in [0, R + 8)
    T k[R + 8];
    T Dk = second_diff(w + 4);
#pragma unroll
    for (int u = 0; u < R + 8; ++u) {
        const T Dk1 = second_diff(w + u + 5);
        const T y = spline(a, b, g, d, w[u + 4], w[u + 5], Dk, Dk1);
        Dk = Dk1;
        const int row = j0 - 4 + u;
        k[u] = (BC == BC_PERIODIC || (row >= 0 && row < np)) ? y : T(0);
    }
    const T cc = (T)c;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T *q = k + r + 4;
        T sm = q[-4] + q[4];
        sm = vfma(T(-8), q[-3] + q[3], sm);
        sm = vfma(T(28), q[-2] + q[2], sm);
        sm = vfma(T(-56), q[-1] + q[1], sm);
        sm = vfma(T(70), q[0], sm);
        const int j = j0 + r;
        if (j < np) fout[(size_t)j * nx + i] = vfma(-cc, sm, q[0]);
    }
}

// ---------------------------------------------------------------------------
// Step 3 fused with the two half drifts that follow it (step 4 and step 1 of
// the next step).  Once the force is known nothing global separates the kick
// of a row from its drifts, so one workgroup kicks the columns its drift
// windows need and drifts the kicked rows straight from LDS: f is read and
// written once for the three sweeps.  The arithmetic of every value is that
// of the separate kick and drifts, so results are identical bit for bit.
//
// Tile: RB consecutive density blocks (16 RB rows) by TW output columns.  The
// first-pass window of row j starts at column i0 + o_j - 8, o_j = m1_j + m2_j
// the sum of the row's two drift offsets; over the tile these windows lie in
// the KW = TW + 18 + SPR kicked columns starting at i0 + kbase (kbase = min_j
// o_j - 8, reduced mod nx on a periodic x axis), row j's window at offset
// krel_j = o_j - min o.  A grid whose tiles need krel > SPR takes the
// separate kernels.
//
// Work per row (one barrier per row, three rows in flight):
//   kick of row r: every lane kicks one column (NT >= KW lanes) from a
//     sliding register window of its column (the kick of row r needs the
//     samples r - 4 + m .. r + 5 + m), loads requested PF rows ahead, and
//     writes the kicked value to slot t of the row's LDS buffer;
//   first half drift of row r - 1 (the first W1 waves): runs of V1 = 5
//     adjacent intermediate values per lane, TW + 9 of them per row;
//   second half drift of row r - 2 (the next W2 waves): runs of V2 = 4
//     outputs per lane, stored to HBM, and their serial column sums over the
//     block (density partial sums).
// A run of V outputs shares its V + 1 stencils (V + 9 samples), so a lane
// computes 1 + 1/V stencils per output instead of 2.
// ---------------------------------------------------------------------------
constexpr int KD_SPR = 8;
// rows per barrier interval of the fused kernel
constexpr int KD_RPI = 2;

// Geometry of a fused tile of TW columns whose rows' windows lie within SPR
// columns of slack: runs of two adjacent values per lane in both half drifts
// (16-byte LDS accesses, conflict-free), W1 waves for the first half drift
// (TW + 9 values per row) and W2 for the second (TW outputs), one kicked
// column per lane over the KW = TW + 18 + SPR columns the windows need.  Every
// wave kicks; TW = 230 (four waves) and 486 (eight) with 8 columns of slack,
// and TW = 182 with 56, make the kicked columns and both half drifts fill
// their waves.
template <int TW, int SPR = KD_SPR>
struct KDGeom {
    static constexpr int V = 2;                          // outputs per lane in the half drifts
    static constexpr int MIDN = TW + 9;                  // first-pass values per row
    static constexpr int NRUN1 = (MIDN + V - 1) / V;     // first-pass lanes
    static constexpr int NRUN2 = TW / V;                 // second-pass lanes
    static constexpr int W1 = (NRUN1 + 63) / 64, W2 = (NRUN2 + 63) / 64;
    static constexpr int KW = TW + 18 + SPR;             // kicked columns per row
    static constexpr int NWK = (KW + 63) / 64;
    static constexpr int NW = NWK > W1 + W2 ? NWK : W1 + W2;  // waves
    static constexpr int NT = 64 * NW;
    // Role of wave w in a workgroup rotated by `rot`: roles [0, W1) run the
    // first half drift, [W1, W1 + W2) the second.  Rotating the roles from one
    // workgroup to the next spreads them over the SIMDs.
    static __device__ __forceinline__ int role(int w, int rot) { return (w + NW - rot) % NW; }
    // kicked row: column c of the range at slot c + (krel & 1), so that every
    // row's window starts at an even slot; both buffers padded for the reads
    // of the last runs (V + 10 values from slot V u)
    static constexpr int NBUF = 2 * KD_RPI;  // rows in each LDS ring
    static constexpr int KLD = NT + 16;
    static constexpr int MLD = NRUN1 * V + 16;
    static_assert(TW % V == 0, "whole second-pass runs");
    static_assert(SPR + 1 + V * (NRUN1 - 1) + V + 10 <= KLD, "first-pass reads stay in the kicked row");
    static_assert(V * (NRUN2 - 1) + V + 10 <= MLD, "second-pass reads stay in the first-pass row");
};

// P2: the calling wave runs the second half drift (and stores); the other
// waves run the first half drift (or only kick).  The two roles are separate
// code, so that the wait of each for its requested kick samples counts only
// its own memory operations.
template <typename T, int BCX, int BCP, int TW, int PF, int RB, bool FULL, bool P2, int SPR = KD_SPR>
__device__ __forceinline__ void kick_drift_tile(const T *__restrict__ fin, T *__restrict__ fout,
                                                const double *__restrict__ F, double dt, double dp,
                                                const int32_t *__restrict__ dm2, const double4 *__restrict__ dw1,
                                                const double4 *__restrict__ dw2, const int32_t *__restrict__ kbase,
                                                const int32_t *__restrict__ krel, double *__restrict__ part, int nx,
                                                int np, int tx, int ty, int rw, T *kbuf, T *mbuf)
{
    using G = KDGeom<TW, SPR>;
    using V2 = typename Vec2<T>::type;
    constexpr int V = G::V, R = ROWS_PER_BLOCK, KLD = G::KLD, MLD = G::MLD;
    constexpr int NS = R + 10 + PF;  // window slots: samples of a block plus those requested ahead
    static_assert(NS <= 32, "one mask bit per sample");
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int i0 = tx * TW;
    const int j0 = ty * (R * RB);
    const int nr = FULL ? R * RB : min(R * RB, np - j0);  // rows of the tile

    // padding of the row buffers (read only by values that are never kept)
    for (int s = G::NT + t; s < KLD; s += G::NT)
#pragma unroll
        for (int b = 0; b < G::NBUF; ++b) kbuf[b * KLD + s] = T(0);
    for (int s = G::NRUN1 * V + t; s < MLD; s += G::NT)
#pragma unroll
        for (int b = 0; b < G::NBUF; ++b) mbuf[b * MLD + s] = T(0);

    // The kicked column of this lane: foot of its p shift (eq. step3), the
    // spline weights, and the element index of its first sample.
    const int cL = i0 + kbase[ty];
    const int c = cL + t;
    int gc;
    bool colin = true;
    if (BCX == BC_PERIODIC) {
        gc = wrap(c, nx);
    } else {
        gc = min(max(c, 0), nx - 1);
        colin = c >= 0 && c < nx;
    }
    // every kicked column lies inside the grid (or the axis is periodic): no mask
    const bool kick_in = BCX == BC_PERIODIC || (cL >= 0 && cL + G::NT <= nx);
    const Foot ft = foot_of_shift((F[gc] * dt) / dp);
    const int m = reduce_offset(ft.m, np, BCP);
    const T ka = (T)ft.a, kb = (T)ft.b, kg = (T)ft.g, kd = (T)ft.d;
    const uint32_t total = (uint32_t)np * (uint32_t)nx;
    // periodic p: element index of the next sample to request (one row per
    // request, wrapped by one subtraction); zero p: row of sample 0
    int rb0 = j0 + m - 4;
    uint32_t nidx = 0;
    if (BCP == BC_PERIODIC) {
        rb0 = wrap(rb0, np);
        nidx = (uint32_t)rb0 * (uint32_t)nx + (uint32_t)gc;
    }
    uint32_t inside = 0;  // zero p: bit s says that sample s lies in the grid
    T w[NS];
    auto request = [&](int s) {
        // sample s of the window (of the current block)
        if (BCP == BC_PERIODIC) {
            w[s] = fin[nidx];
            nidx += (uint32_t)nx;
            nidx = min(nidx, nidx - total);  // unsigned: subtracts total once past the end
        } else {
            const int q = rb0 + s;
            inside |= (uint32_t)(q >= 0 && q < np) << s;
            w[s] = fin[(size_t)min(max(q, 0), np - 1) * (size_t)nx + (size_t)gc];
        }
    };
    auto settle = [&](int s) {
        if (BCP != BC_PERIODIC) w[s] = (inside >> s & 1u) ? w[s] : T(0);
    };
#pragma unroll
    for (int s = 0; s < 10 + PF; ++s) request(s);
#pragma unroll
    for (int s = 0; s < 9; ++s) settle(s);
    T Dk = second_diff(w + 4);

    const bool pass1 = !P2 && rw < G::W1;
    const int u1 = 64 * rw + lane, u2 = 64 * (rw - G::W1) + lane;  // run of the lane in its pass
    const int i = i0 + V * u2;  // first output column of a second-pass lane
    const bool own2 = P2 && u2 < G::NRUN2 && i < nx;
    const bool own1 = pass1 && u1 < G::NRUN1;

    // Interval it of block blk kicks rows P it .. P it + P - 1 of the block
    // (P = KD_RPI rows per barrier interval), runs the first half drift of the
    // P rows before them and the second of the P rows before those; negative
    // rows are the previous block's last ones, so the pipeline runs on across
    // the blocks of a tile and only the last block drains it (two more
    // intervals).  Row q's buffers are slot q mod 2P of each ring.
    constexpr int P = KD_RPI, NI = R / P, NB = G::NBUF;
    static_assert(R % P == 0 && (NB & (NB - 1)) == 0, "whole intervals per block, ring of 2^k rows");
    double acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = 0.0;
#pragma unroll
    for (int blk = 0; blk < RB; ++blk) {
        const int jb = j0 + R * blk;
        if (!FULL && R * blk >= nr) break;  // uniform
        const bool lastb = blk + 1 == RB || (!FULL && R * (blk + 1) >= nr);  // uniform
#pragma unroll
        for (int it = 0; it < NI + 2; ++it) {
            if (it >= NI && !lastb) break;  // uniform
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int r = P * it + s;
                if (it < NI && (FULL || R * blk + r < nr)) {
                    // kick of row r into its buffer
                    settle(r + 9);
                    const T Dk1 = second_diff(w + r + 5);
                    T y = spline(ka, kb, kg, kd, w[r + 4], w[r + 5], Dk, Dk1);
                    Dk = Dk1;
                    if (!kick_in) y = colin ? y : T(0);
                    kbuf[(r & (NB - 1)) * KLD + (krel[jb + r] & 1) + t] = y;
                    // samples of the next block are requested too (the last
                    // block's extra requests read valid rows and are unused)
                    if (r + 10 + PF < NS && (RB > 1 || r + 10 + PF < R + 10)) request(r + 10 + PF);
                }
            }
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int q1 = P * (it - 1) + s;
                if (!P2 && (it >= 1 || blk > 0) && it - 1 < NI && (FULL || R * blk + q1 < nr) && own1) {
                    // first half drift (table 1) of row q1 at the positions
                    // i0 + m2 - 4 + q, q in [0, TW + 9), that the second reads
                    const int j = jb + q1;
                    const int rel = krel[j];
                    const T *src = kbuf + (q1 & (NB - 1)) * KLD + rel + (rel & 1);
                    const double4 w1 = dw1[j];
                    T o[V];
                    spline_run<T, V>(src, u1, (T)w1.x, (T)w1.y, (T)w1.z, (T)w1.w, o);
                    if (BCX == BC_ZERO) {
                        const int lo = i0 + dm2[j] - 4;  // position of first-pass value 0
                        if (!(lo >= 0 && lo + G::MIDN <= nx)) {
                            const int q = lo + V * u1;
#pragma unroll
                            for (int k = 0; k < V; ++k)
                                if (q + k < 0 || q + k >= nx) o[k] = T(0);
                        }
                    }
                    V2 ww;
                    ww.x = o[0];
                    ww.y = o[1];
                    reinterpret_cast<V2 *>(mbuf + (q1 & (NB - 1)) * MLD)[u1] = ww;
                }
            }
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int q2 = P * (it - 2) + s;
                if (P2 && (it >= 2 || blk > 0) && (FULL || R * blk + q2 < nr) && own2) {
                    // second half drift (table 2) of row q2: outputs i, i + 1
                    const int j = jb + q2;
                    const double4 wd = dw2[j];
                    T o[V];
                    spline_run<T, V>(mbuf + (q2 & (NB - 1)) * MLD, u2, (T)wd.x, (T)wd.y, (T)wd.z, (T)wd.w, o);
                    if (FULL) {
                        V2 ww;
                        ww.x = o[0];
                        ww.y = o[1];
                        *reinterpret_cast<V2 *>(fout + (size_t)j * nx + i) = ww;
                    } else {
                        store_run<T, V>(fout + (size_t)j * nx, i, nx, o);
                    }
#pragma unroll
                    for (int k = 0; k < V; ++k) acc[k] = acc[k] + (double)o[k];
                }
            }
            if (P2 && it == 1 && blk > 0) {
                // the previous block's sums are complete
                if (own2) {
                    double *prow = part + (size_t)(ty * RB + blk - 1) * nx;
#pragma unroll
                    for (int k = 0; k < V; ++k)
                        if (i + k < nx) prow[i + k] = acc[k];
                }
#pragma unroll
                for (int k = 0; k < V; ++k) acc[k] = 0.0;
            }
            __syncthreads();
        }
        if (P2 && own2 && lastb) {
            double *prow = part + (size_t)(ty * RB + blk) * nx;
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (i + k < nx) prow[i + k] = acc[k];
        }
        // slide the window by one block: sample s + 16 becomes sample s
        if (RB > 1) {
#pragma unroll
            for (int s = 0; s + R < NS; ++s) w[s] = w[s + R];
            inside >>= R;
            rb0 += R;
        }
    }
}

template <typename T, int BCX, int BCP, int TW, int PF, int RB>
static __global__ __launch_bounds__(KDGeom<TW>::NT) void k_kick_drift(
    const T *__restrict__ fin, T *__restrict__ fout, const double *__restrict__ F, double dt, double dp,
    const int32_t *__restrict__ dm2, const double4 *__restrict__ dw1, const double4 *__restrict__ dw2,
    const int32_t *__restrict__ kbase, const int32_t *__restrict__ krel, double *__restrict__ part, int nx, int np,
    int ntx, int nty)
{
    using G = KDGeom<TW>;
    __shared__ __attribute__((aligned(16))) T kbuf[G::NBUF * G::KLD];  // ring of kicked rows
    __shared__ __attribute__((aligned(16))) T mbuf[G::NBUF * G::MLD];  // ring of first-pass rows
    int tx, ty;
    if (!xcd_tile(ntx, nty, tx, ty)) return;
    // every row of the tile in the grid, and rows of an even length (aligned
    // two-value stores)
    const bool full = (ty + 1) * (ROWS_PER_BLOCK * RB) <= np && (nx & 1) == 0;
    const int rw = G::role(threadIdx.x >> 6, blockIdx.x % G::NW);
    const bool p2 = rw >= G::W1 && rw < G::W1 + G::W2;
#define KDT(FL, P)                                                                                                  \
    kick_drift_tile<T, BCX, BCP, TW, PF, RB, FL, P>(fin, fout, F, dt, dp, dm2, dw1, dw2, kbase, krel, part, nx, np, tx, \
                                                    ty, rw, kbuf, mbuf)
    if (full) {
        if (p2)
            KDT(true, true);
        else
            KDT(true, false);
    } else {
        if (p2)
            KDT(false, true);
        else
            KDT(false, false);
    }
#undef KDT
}

// ---------------------------------------------------------------------------
// Eq. (tridiagsys): the global spline, the paper's baseline for the local f''.
// D_i = f''_i du^2 solves D_{i-1} + 4 D_i + D_{i+1} = 6 S_i with S_i =
// f_{i+1} - 2 f_i + f_{i-1} (on a periodic line, or on the line continued by
// zeros).  The (1, 4, 1) operator factors as -(1/r)(1 - r E)(1 - r E^-1),
// E the shift to the next node and r = sqrt(3) - 2 its root inside the unit
// circle, so D = -6 r x with y_i = S_i + r y_{i-1} (causal) and x_i = y_i +
// r x_{i+1} (anticausal): the convolution of S with sqrt(3) r^|k|.  Each
// thread runs both recursions over a chunk of GS_CH nodes, started GS_K nodes
// outside its chunk from 0 (|r|^GS_K is below FP64 resolution), so the
// chunks need no sequential pass.  On a periodic line the recursions wrap;
// with zero extension they run over the line continued by GS_E zeros at each
// end, where D decays by |r| per cell (farther feet read D = 0).  One
// workgroup of 256 threads moves one line of n <= GS_MAX_N samples through
// LDS (the samples, and S, y and D in turn in a second array), then
// evaluates the spline of eq. (splinegen) at the feet.  Lines are the rows
// of f (the drift) or of its transpose (the kick, shift from the force of
// the column).
// ---------------------------------------------------------------------------
constexpr int GS_K = 30, GS_E = GS_K + 2, GS_MAX_N = 4096, GS_NT = 256;
constexpr int GS_LDS = GS_MAX_N + 2 * GS_E;
constexpr int GS_CH = (GS_LDS + GS_NT - 1) / GS_NT;  // nodes per thread

template <typename T, int BC, bool KICK>
static __global__ __launch_bounds__(GS_NT) void k_gs_line(const T *__restrict__ fin, T *__restrict__ fout, int n,
                                                   const int32_t *__restrict__ dm,
                                                   const double4 *__restrict__ dw,
                                                   const double *__restrict__ F, double dt, double dh,
                                                   const double *__restrict__ gcoef)
{
    __shared__ T fe[GS_LDS], Q[GS_LDS];
    const int line = blockIdx.x, t = threadIdx.x;
    const T *src = fin + (size_t)line * n;
    const T r = (T)gcoef[0], cD = (T)gcoef[1];
    // working line: the n nodes (periodic, indices mod n) or the extended
    // line e = i + GS_E, i in [-GS_E, n + GS_E) (zero extension)
    const int N = BC == BC_PERIODIC ? n : n + 2 * GS_E;
    {
        // all GS_CH loads of a thread in flight at once
        T v[GS_CH];
#pragma unroll
        for (int u = 0; u < GS_CH; ++u) {
            const int e = t + u * GS_NT;
            const int i = BC == BC_PERIODIC ? e : e - GS_E;
            v[u] = src[min(max(i, 0), n - 1)];
        }
#pragma unroll
        for (int u = 0; u < GS_CH; ++u) keep_issued(v[u]);
#pragma unroll
        for (int u = 0; u < GS_CH; ++u) {
            const int e = t + u * GS_NT;
            const int i = BC == BC_PERIODIC ? e : e - GS_E;
            if (e < N) fe[e] = (i >= 0 && i < n) ? v[u] : T(0);
        }
    }
    __syncthreads();
    // a[e] under the boundary rule of the working line; e lies in
    // [-GS_K, N + GS_K + GS_CH), so two conditional steps wrap it once the
    // line is longer than that excursion (shorter lines take the division)
    const bool short_line = n < GS_K + GS_CH + 1;
    auto at = [&](const T *a, int e) -> T {
        if (BC == BC_PERIODIC) {
            if (short_line) return a[wrap(e, n)];
            const int q = e < 0 ? e + n : e;
            return a[q >= n ? q - n : q];
        }
        return (e >= 0 && e < N) ? a[e] : T(0);
    };
    for (int e = t; e < N; e += GS_NT)
        Q[e] = (BC != BC_PERIODIC && (e == 0 || e == N - 1)) ? T(0)
                                                             : (at(fe, e - 1) + at(fe, e + 1)) - T(2) * fe[e];
    __syncthreads();
    const int c0 = t * GS_CH;  // this thread's chunk [c0, c0 + GS_CH)
    const bool mine = c0 < N;
    T w[GS_CH];
    if (mine) {  // causal recursion y_e = S_e + r y_{e-1}
        T acc = T(0);
        for (int k = GS_K; k >= 1; --k) acc = vfma(r, acc, at(Q, c0 - k));
#pragma unroll
        for (int u = 0; u < GS_CH; ++u) {
            acc = vfma(r, acc, at(Q, c0 + u));
            w[u] = acc;
        }
    }
    __syncthreads();
    if (mine)
#pragma unroll
        for (int u = 0; u < GS_CH; ++u)
            if (c0 + u < N) Q[c0 + u] = w[u];
    __syncthreads();
    if (mine) {  // anticausal recursion x_e = y_e + r x_{e+1}, D = -6 r x
        T acc = T(0);
        for (int k = GS_K + GS_CH - 1; k >= GS_CH; --k) acc = vfma(r, acc, at(Q, c0 + k));
#pragma unroll
        for (int u = GS_CH - 1; u >= 0; --u) {
            acc = vfma(r, acc, at(Q, c0 + u));
            w[u] = cD * acc;
        }
    }
    __syncthreads();
    if (mine)
#pragma unroll
        for (int u = 0; u < GS_CH; ++u)
            if (c0 + u < N) Q[c0 + u] = w[u];
    __syncthreads();
    // foot of the line's shift
    int m;
    T a, b, gg, d;
    if (KICK) {
        const Foot ft = foot_of_shift((F[line] * dt) / dh);
        m = reduce_offset(ft.m, n, BC);
        a = (T)ft.a;
        b = (T)ft.b;
        gg = (T)ft.g;
        d = (T)ft.d;
    } else {
        m = dm[line];
        const double4 wv = dw[line];
        a = (T)wv.x;
        b = (T)wv.y;
        gg = (T)wv.z;
        d = (T)wv.w;
    }
    T *dst = fout + (size_t)line * n;
    for (int i = t; i < n; i += GS_NT) {
        const int k = i + m;  // cell [k, k + 1]
        T fk, fk1, Dk, Dk1;
        if (BC == BC_PERIODIC) {
            const int q = k >= n ? k - n : k, q1 = q + 1 == n ? 0 : q + 1;  // m in [0, n)
            fk = fe[q];
            fk1 = fe[q1];
            Dk = Q[q];
            Dk1 = Q[q1];
        } else {
            fk = (k >= 0 && k < n) ? fe[k + GS_E] : T(0);
            fk1 = (k + 1 >= 0 && k + 1 < n) ? fe[k + 1 + GS_E] : T(0);
            Dk = (k > -GS_E && k < n + GS_E - 1) ? Q[k + GS_E] : T(0);
            Dk1 = (k + 1 > -GS_E && k + 1 < n + GS_E - 1) ? Q[k + 1 + GS_E] : T(0);
        }
        dst[i] = spline(a, b, gg, d, fk, fk1, Dk, Dk1);
    }
}

// Transpose of an rows x cols array through 64 x 64 LDS tiles (the kick of
// the global spline runs on the rows of the transpose).
template <typename T>
static __global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ in, T *__restrict__ out, int rows,
                                                   int cols)
{
    __shared__ T tile[64][65];
    const int tcols = (cols + 63) / 64;
    const int bx = blockIdx.x % tcols, by = blockIdx.x / tcols;
    const int c0 = bx * 64, r0 = by * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4)
        if (r0 + r < rows && c0 + tx < cols) tile[r][tx] = in[(size_t)(r0 + r) * cols + c0 + tx];
    __syncthreads();
    for (int c = ty; c < 64; c += 4)
        if (c0 + c < cols && r0 + tx < rows) out[(size_t)(c0 + c) * rows + r0 + tx] = tile[tx][c];
}

// Density partial sums of f (serial over the rows of each 16-row block, in
// the order the drift kernels accumulate them).
template <typename T>
static __global__ __launch_bounds__(256) void k_partials(const T *__restrict__ f, double *__restrict__ part, int nx,
                                                  int np)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    const int b = blockIdx.y;
    const int jend = min(b * ROWS_PER_BLOCK + ROWS_PER_BLOCK, np);
    double acc = 0.0;
    for (int j = b * ROWS_PER_BLOCK; j < jend; ++j) acc = acc + (double)f[(size_t)j * nx + i];
    part[(size_t)b * nx + i] = acc;
}

// ---------------------------------------------------------------------------
// Density rho_i = dp * sum_j f_ji from the 16-row partial sums.  One
// workgroup per 16 columns: thread (c, g) forms the serial sums of the block
// classes l = g, g + 16, g + 32, g + 48 (blocks b = l mod 64, ascending b) of
// column c, so that a wavefront load reads 16 adjacent columns of 4 block
// rows; the 64 class sums of a column are then combined by the pairwise tree
// in LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void density_block(const double *__restrict__ part, double *__restrict__ rho, int nx,
                                              int nblk, double dp, int blk, double (*S)[17])
{
    const int c = threadIdx.x & 15;
    const int g = threadIdx.x >> 4;
    const int i = blk * 16 + c;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < nx) {
        for (int b0 = 0; b0 < nblk; b0 += 64) {
            double x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int b = b0 + g + 16 * k;
                x[k] = b < nblk ? part[(size_t)b * nx + i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (b0 + g + 16 * k < nblk) acc[k] = acc[k] + x[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) S[g + 16 * k][c] = acc[k];
    __syncthreads();
    for (int d = 32; d >= 1; d >>= 1) {
        for (int k = threadIdx.x; k < d * 16; k += 256) {
            const int l = k >> 4, cc = k & 15;
            S[l][cc] = S[l][cc] + S[l + d][cc];
        }
        __syncthreads();
    }
    if (g == 0 && i < nx) rho[i] = dp * S[0][c];
}


// The same sums with 1024 threads: thread (c, g) forms the serial sum of
// block class g alone, its loads (blocks g, g + 64, g + 128, g + 192 of a
// round) all in flight at once; then wavefront c folds the 64 class sums of
// column c with the xor butterfly (the same association as the pairwise tree
// S[g] + S[g + d], d = 32, ..., 1: addition is commutative).
static __global__ __launch_bounds__(1024) void k_density(const double *__restrict__ part, double *__restrict__ rho,
                                                  int nx, int nblk, double dp)
{
    __shared__ double S[16][65];
    const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + c;
    const int ic = min(i, nx - 1);
    double acc = 0.0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        double x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = part[(size_t)min(b0 + g + 64 * k, nblk - 1) * nx + ic];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) keep_issued(x[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (b0 + g + 64 * k < nblk) acc = acc + x[k];
    }
    S[c][g] = acc;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double v = wave_sum(S[w][lane]);
    const int io = blockIdx.x * 16 + w;
    if (lane == 0 && io < nx) rho[io] = dp * v;
}

// Stage two arrays of n doubles into LDS (whole workgroup), the sixteen loads
// of a round per thread in flight before their LDS writes.
__device__ __forceinline__ void stage2(double *d0, const double *__restrict__ s0, double *d1,
                                       const double *__restrict__ s1, int n)
{
    const int bd = blockDim.x;
    for (int k0 = threadIdx.x; k0 < n; k0 += 8 * bd) {
        double v[2][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = min(k0 + u * bd, n - 1);
            v[0][u] = s0[k];
            v[1][u] = s1[k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            keep_issued(v[0][u]);
            keep_issued(v[1][u]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + u * bd < n) {
                d0[k0 + u * bd] = v[0][u];
                d1[k0 + u * bd] = v[1][u];
            }
    }
}

// Stage three arrays of n doubles into LDS (whole workgroup), the twelve
// loads of a round per thread in flight before their LDS writes.
__device__ __forceinline__ void stage3(double *d0, const double *__restrict__ s0, double *d1,
                                       const double *__restrict__ s1, double *d2, const double *__restrict__ s2, int n)
{
    const int bd = blockDim.x;
    for (int k0 = threadIdx.x; k0 < n; k0 += 4 * bd) {
        double v[3][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = min(k0 + u * bd, n - 1);
            v[0][u] = s0[k];
            v[1][u] = s1[k];
            v[2][u] = s2[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            keep_issued(v[0][u]);
            keep_issued(v[1][u]);
            keep_issued(v[2][u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k0 + u * bd < n) {
                d0[k0 + u * bd] = v[0][u];
                d1[k0 + u * bd] = v[1][u];
                d2[k0 + u * bd] = v[2][u];
            }
    }
}

// Magnetization of eq. (mxmydef) by one wavefront from LDS copies of rho, cos
// and sin; every lane returns (mx, my).
__device__ inline void magnetization(const double *rho, const double *cs, const double *sn, int n, double dx,
                                     double &mx, double &my)
{
    const int lane = threadIdx.x & 63;
    double c = 0.0, s = 0.0;
    int i = lane;
    // eight terms of each chain requested at once (the chains stay in order)
    for (; i + 7 * 64 < n; i += 8 * 64) {
        double cv[8], sv[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            cv[u] = cs[i + 64 * u];
            sv[u] = sn[i + 64 * u];
            rv[u] = rho[i + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c = fma(cv[u], rv[u], c);
            s = fma(sv[u], rv[u], s);
        }
    }
    for (; i < n; i += 64) {
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

constexpr int FORCE_LDS_MAX = 4096;  // nx up to which rho, cos, sin are staged in LDS

// HMF force, eq. (hmfmeanforce): F_i = -sin(x_i) M_x + cos(x_i) M_y.  One
// workgroup; wavefront 0 forms (M_x, M_y).  L: 3 SMAX doubles (STAGED, n <= SMAX).
template <bool STAGED, int SMAX = FORCE_LDS_MAX>
__device__ __forceinline__ void force_hmf_block(const double *__restrict__ rho, const double *__restrict__ cs,
                                                const double *__restrict__ sn, double *__restrict__ F, int n,
                                                double dx, double *mxmy, double *hist, int64_t *hcount, int64_t hcap,
                                                double *L, double *M)
{
    const double *r = rho, *c = cs, *s = sn;
    if (STAGED) {
        stage3(L, rho, L + SMAX, cs, L + 2 * SMAX, sn, n);
        __syncthreads();
        r = L;
        c = L + SMAX;
        s = L + 2 * SMAX;
    }
    if (threadIdx.x < 64) {
        double mx, my;
        magnetization(r, c, s, n, dx, mx, my);
        if (threadIdx.x == 0) {
            M[0] = mx;
            M[1] = my;
            record_history(mxmy, hist, hcount, hcap, mx, my);
        }
    }
    __syncthreads();
    const double mx = M[0], my = M[1];
    for (int i = threadIdx.x; i < n; i += blockDim.x) F[i] = fma(my, c[i], -(mx * s[i]));
}

// The single-grid form: wavefront 0 forms (M_x, M_y) from the arrays in
// memory (the same chains as magnetization()), then every thread writes its
// forces; no staging of the three arrays.
static __global__ __launch_bounds__(1024) void k_force_hmf(const double *__restrict__ rho, const double *__restrict__ cs,
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

// Magnetization only (ring model, batched force phase).  One workgroup,
// wavefront 0 reduces.  L: 3 SMAX doubles (STAGED, n <= SMAX).
template <bool STAGED, int SMAX = FORCE_LDS_MAX>
__device__ __forceinline__ void magnetization_block(const double *__restrict__ rho, const double *__restrict__ cs,
                                                    const double *__restrict__ sn, int n, double dx, double *mxmy,
                                                    double *hist, int64_t *hcount, int64_t hcap, double *L)
{
    const double *r = rho, *c = cs, *s = sn;
    if (STAGED) {
        stage3(L, rho, L + SMAX, cs, L + 2 * SMAX, sn, n);
        __syncthreads();
        r = L;
        c = L + SMAX;
        s = L + 2 * SMAX;
    }
    if (threadIdx.x < 64) {
        double mx, my;
        magnetization(r, c, s, n, dx, mx, my);
        if (threadIdx.x == 0) record_history(mxmy, hist, hcount, hcap, mx, my);
    }
}

// Ring force, eq. (meanforce) with eq. (ringpot): F_i = -dx sum_k K_{(i-k)
// mod n} rho_k with K the tabulated V'.  One wavefront per output i.
__device__ __forceinline__ void force_ring_output(const double *__restrict__ rho, const double *__restrict__ K,
                                                  double *__restrict__ F, int n, double dx, int i)
{
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    int k = lane;
    // eight terms of the chain requested at once (the chain stays in order)
    for (; k + 7 * 64 < n; k += 8 * 64) {
        double kv[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            int d = i - (k + 64 * u);
            if (d < 0) d += n;
            kv[u] = K[d];
            rv[u] = rho[k + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(kv[u], rv[u], acc);
    }
    for (; k < n; k += 64) {
        int d = i - k;
        if (d < 0) d += n;
        acc = fma(K[d], rho[k], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) F[i] = -(dx * acc);
}

// Workgroup 0 forms the magnetization (M_x, M_y) for the history instead (the
// ring force does not use it), dispatched first so that its chain overlaps
// the outputs' workgroups.  STAGED (n <= RING_LDS_MAX): every workgroup first
// copies the arrays it reads (rho and K; rho, cos and sin for workgroup 0)
// into LDS, whose reads in the chains are conflict-free (adjacent lanes,
// adjacent words), and its four wavefronts then form RING_OUT_WG / 4 outputs
// each; otherwise one output per wavefront straight from global memory.
// Launch 1 + ceil(n / ring_outputs_per_wg(n)) workgroups of 256 threads.
constexpr int RING_LDS_MAX = 2048;
constexpr int RING_OUT_WG = 8;
__host__ __device__ constexpr int ring_outputs_per_wg(int n) { return n <= RING_LDS_MAX ? RING_OUT_WG : 4; }

template <bool STAGED>
static __global__ __launch_bounds__(256) void k_force_ring(const double *__restrict__ rho, const double *__restrict__ K,
                                                    double *__restrict__ F, int n, double dx,
                                                    const double *__restrict__ cs, const double *__restrict__ sn,
                                                    double *mxmy, double *hist, int64_t *hcount, int64_t hcap)
{
    __shared__ double L[STAGED ? 3 * RING_LDS_MAX : 1];
    if (blockIdx.x == 0) {
        const double *r = rho, *c = cs, *s = sn;
        if (STAGED) {
            stage3(L, rho, L + RING_LDS_MAX, cs, L + 2 * RING_LDS_MAX, sn, n);
            __syncthreads();
            r = L;
            c = L + RING_LDS_MAX;
            s = L + 2 * RING_LDS_MAX;
        }
        if (threadIdx.x < 64) {
            double mx, my;
            magnetization(r, c, s, n, dx, mx, my);
            if (threadIdx.x == 0) record_history(mxmy, hist, hcount, hcap, mx, my);
        }
        return;
    }
    constexpr int OUT = STAGED ? RING_OUT_WG : 4;
    const double *r = rho, *k = K;
    if (STAGED) {
        stage2(L, rho, L + RING_LDS_MAX, K, n);
        __syncthreads();
        r = L;
        k = L + RING_LDS_MAX;
    }
#pragma unroll
    for (int q = 0; q < OUT / 4; ++q) {
        const int i = (blockIdx.x - 1) * OUT + (threadIdx.x >> 6) * (OUT / 4) + q;
        if (i < n) force_ring_output(r, k, F, n, dx, i);
    }
}

// Sheet force, eq. (sheetpot) with V = 2 pi G |x|: F_i = K (S - 2 P_i - rho_i),
// K = 2 pi G dx, P_i the exclusive prefix sum of rho and S its total.
// Wavefront 0 scans: lane l owns the contiguous chunk [l c, (l+1) c),
// c = ceil(n/64); chunk totals by an inclusive Hillis-Steele scan
// d = 1, 2, ..., 32.  When staged, rho is held in LDS chunk-transposed
// (element l c + k at k 65 + l) so that the 64 lanes walking their chunks read
// adjacent words; F is written back in place and stored coalesced.
constexpr int SHEET_LDS_MAX = 16384;
constexpr int SHEET_LDS_WORDS = (SHEET_LDS_MAX / 64) * 65;

template <bool STAGED>
__device__ __forceinline__ void force_sheet_block(const double *__restrict__ rho, double *__restrict__ F, int n,
                                                  double K, double *L)
{
    const int c = (n + 63) / 64;
    if (STAGED) {
        const int bd = blockDim.x;
        for (int i0 = threadIdx.x; i0 < n; i0 += 4 * bd) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = rho[min(i0 + u * bd, n - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) keep_issued(v[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * bd;
                if (i < n) L[(i % c) * 65 + i / c] = v[u];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        const int len = min(c, n - l * c);  // <= 0 past the end
        double tot = 0.0;
        int k = 0;
        // sixteen samples requested at once, summed in order
        for (; k + 16 <= len; k += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = STAGED ? L[(k + u) * 65 + l] : rho[l * c + k + u];
#pragma unroll
            for (int u = 0; u < 16; ++u) tot = tot + v[u];
        }
        for (; k < len; ++k) tot = tot + (STAGED ? L[k * 65 + l] : rho[l * c + k]);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double v = __shfl_up(tot, d, 64);
            if (l >= d) tot = v + tot;
        }
        double excl = __shfl_up(tot, 1, 64);
        if (l == 0) excl = 0.0;
        const double S = __shfl(tot, 63, 64);
        double acc = 0.0;
        auto one = [&](int kk, double r) {
            const double Pi = excl + acc;
            const double f = K * (fma(-2.0, Pi, S) - r);
            if (STAGED)
                L[kk * 65 + l] = f;
            else
                F[l * c + kk] = f;
            acc = acc + r;
        };
        k = 0;
        for (; k + 16 <= len; k += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = STAGED ? L[(k + u) * 65 + l] : rho[l * c + k + u];
#pragma unroll
            for (int u = 0; u < 16; ++u) one(k + u, v[u]);
        }
        for (; k < len; ++k) one(k, STAGED ? L[k * 65 + l] : rho[l * c + k]);
    }
    if (STAGED) {
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) F[i] = L[(i % c) * 65 + i / c];
    }
}

template <bool STAGED>
static __global__ __launch_bounds__(1024) void k_force_sheet(const double *__restrict__ rho, double *__restrict__ F, int n,
                                                      double K)
{
    __shared__ double L[STAGED ? SHEET_LDS_WORDS : 1];
    force_sheet_block<STAGED>(rho, F, n, K, L);
}

// ---------------------------------------------------------------------------
// Diagnostics.  Pass 1: 16-row block sums of f, p f, p^2/2 f and f^2.
// ---------------------------------------------------------------------------
template <typename T>
static __global__ __launch_bounds__(256) void k_mom_blocks(const T *__restrict__ f, double *__restrict__ scratch, int nx,
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

// Pass 1b: 16-row block sums of f log f over f > 0 (entropy density) and of
// f over f < 0 (negative mass), into planes 0 and 1 of the scratch.
template <typename T>
static __global__ __launch_bounds__(256) void k_mom_blocks2(const T *__restrict__ f, double *__restrict__ scratch,
                                                     int nx, int np, int nblk)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    const int b = blockIdx.y;
    const int j0 = b * ROWS_PER_BLOCK;
    const int jend = min(j0 + ROWS_PER_BLOCK, np);
    double se = 0.0, sn = 0.0;
    for (int j = j0; j < jend; ++j) {
        const double v = (double)f[(size_t)j * nx + i];
        se = se + (v > 0.0 ? v * log(v) : 0.0);
        sn = sn + (v < 0.0 ? v : 0.0);
    }
    const size_t plane = (size_t)nblk * nx;
    const size_t o = (size_t)b * nx + i;
    scratch[o] = se;
    scratch[plane + o] = sn;
}

// Pass 2: column quantities col[q0 + q][i] = dp * sum over blocks of scratch
// plane q < nq (one wavefront per column).
static __global__ __launch_bounds__(256) void k_mom_cols(const double *__restrict__ scratch, double *__restrict__ col,
                                                  int nx, int nblk, double dp, int nq, int q0)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nx) return;
    const size_t plane = (size_t)nblk * nx;
    for (int q = 0; q < nq; ++q) {
        double acc = 0.0;
        for (int b = lane; b < nblk; b += 64) acc = acc + scratch[q * plane + (size_t)b * nx + i];
        acc = wave_sum(acc);
        if (lane == 0) col[(size_t)(q0 + q) * nx + i] = dp * acc;
    }
}

// Pass 3 (ring and sheet): phi_i = sum_k V(x_i - x_k) rho_k with V the
// tabulated ring potential, or |i - k| (sheet, in cells).
template <bool RING>
static __global__ __launch_bounds__(256) void k_mom_phi(const double *__restrict__ rho, const double *__restrict__ V,
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
// energy, mx, my, l2, entropy, negative mass}.
static __global__ __launch_bounds__(64) void k_mom_final(const double *__restrict__ col, const double *__restrict__ phi,
                                                  const double *__restrict__ cs, const double *__restrict__ sn,
                                                  double *__restrict__ out, int n, double dx, int model,
                                                  double wcoef)
{
    const int lane = threadIdx.x;
    const double *rho = col, *jj = col + n, *kk = col + 2 * n, *qq = col + 3 * n, *ee = col + 4 * n,
                 *nn = col + 5 * n;
    double sm = 0.0, sj = 0.0, sk = 0.0, sq = 0.0, se = 0.0, sneg = 0.0, c = 0.0, s = 0.0, w = 0.0;
    const bool angular = (model == 0 || model == 1);
    const bool pair = (model == 1 || model == 2);
    for (int i = lane; i < n; i += 64) {
        sm = sm + rho[i];
        sj = sj + jj[i];
        sk = sk + kk[i];
        sq = sq + qq[i];
        se = se + ee[i];
        sneg = sneg + nn[i];
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
    se = wave_sum(se);
    sneg = wave_sum(sneg);
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
        out[8] = -(dx * se);
        out[9] = dx * sneg;
    }
}

// ---------------------------------------------------------------------------
// Batches: many grids (of one storage type) stepped together, one persistent
// launch per phase.  A grid is described by a GridDesc; a cycle (drift,
// density, force, kick) by a Cycle listing the member grids, what each does in
// that cycle and the prefix offsets of their work items.  Workgroups stride
// over the work items of all members; per-grid arithmetic is exactly that of
// the single-grid kernels, whatever workgroup processes a tile.
// ---------------------------------------------------------------------------
constexpr int BATCH_MAX = 256;

enum { DRIFT_NONE = 0, DRIFT_FIRST = 1, DRIFT_PAIR = 2, DRIFT_LAST = 3 };

struct GridDesc {
    void *f[2];
    const int32_t *dm;
    const double4 *dw;
    double *part, *rho, *F;
    const double *Fkick;  // force read by the kick (F, or the EXTERNAL table)
    const double *cs, *sn, *K;
    double *mxmy, *hist;
    int64_t *hcount;
    int64_t hcap;
    int32_t nx, np, nblk, model, bc_x, bc_p;
    int32_t kd_wide;  // fused kick and drift on the wide-slack tiles
    double dx, dp, dt, sheetK;
    const int32_t *kbase, *krel;  // fused kick and drift: tables of the member's 16-row tiles
};

struct Cycle {
    int32_t n;                   // members in this cycle
    int32_t slot[BATCH_MAX];     // GridDesc index of member a
    int8_t drift[BATCH_MAX];     // DRIFT_* (FIRST and PAIR also write density partial sums)
    int8_t kick[BATCH_MAX];      // density, force and kick in this cycle
    int8_t cur[BATCH_MAX];       // current f buffer at the start of the cycle
    int8_t kin[BATCH_MAX];       // f buffer the kick (or fused kick and drift) reads
    int8_t pad[4];
    // work items of the phases: drift tiles, density blocks, force items,
    // tiles of the separate kick, tiles of the fused kick and two half drifts
    int32_t off_drift[BATCH_MAX + 1], off_dens[BATCH_MAX + 1], off_force[BATCH_MAX + 1], off_kick[BATCH_MAX + 1],
        off_kd[BATCH_MAX + 1];
};

// Member owning work item e: the last a with off[a] <= e (off[0] = 0 <= e < off[n]).
__device__ __forceinline__ int find_member(const int32_t *off, int n, int e)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= e)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename T, int NT, int V, int PF>
static __global__ __launch_bounds__(NT) void kb_drift(const GridDesc *__restrict__ gd, const Cycle *__restrict__ cy)
{
    using G1 = DriftGeom<1, NT, V, 0>;
    using G2 = DriftGeom<2, NT, V, 0>;
    constexpr int LDA = G1::LDA > G2::LDA ? G1::LDA : G2::LDA;
    __shared__ __attribute__((aligned(16))) T win[2][LDA];
    __shared__ __attribute__((aligned(16))) T mid[G2::LDM];
    const int n = cy->n;
    const int total = cy->off_drift[n];
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int a = find_member(cy->off_drift, n, e);
        const GridDesc &g = gd[cy->slot[a]];
        const int kind = cy->drift[a], cur = cy->cur[a];
        const int li = e - cy->off_drift[a];
        const int ntx = (g.nx + G1::TW - 1) / G1::TW;
        const int tx = li % ntx, ty = li / ntx;
        const T *fin = (const T *)g.f[cur];
        T *fout = (T *)g.f[cur ^ 1];
        __syncthreads();
#define BD(NP, BC, PT)                                                                                               \
    drift_tile_any<T, NP, BC, PT, NT, V, 0, PF>(fin, fout, g.dm, g.dw, g.dm, g.dw, g.part, g.nx, g.np, tx, ty, win[0],   \
                                                win[1], mid)
        if (g.bc_x == BC_PERIODIC) {
            if (kind == DRIFT_PAIR)
                BD(2, BC_PERIODIC, true);
            else if (kind == DRIFT_FIRST)
                BD(1, BC_PERIODIC, true);
            else
                BD(1, BC_PERIODIC, false);
        } else {
            if (kind == DRIFT_PAIR)
                BD(2, BC_ZERO, true);
            else if (kind == DRIFT_FIRST)
                BD(1, BC_ZERO, true);
            else
                BD(1, BC_ZERO, false);
        }
#undef BD
    }
}

static __global__ __launch_bounds__(256) void kb_density(const GridDesc *__restrict__ gd, const Cycle *__restrict__ cy)
{
    __shared__ double S[64][17];
    const int n = cy->n;
    const int total = cy->off_dens[n];
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int a = find_member(cy->off_dens, n, e);
        const GridDesc &g = gd[cy->slot[a]];
        __syncthreads();
        density_block(g.part, g.rho, g.nx, g.nblk, g.dp, e - cy->off_dens[a], S);
    }
}

// Work items per member: HMF and sheet one workgroup; ring ceil(nx/16)
// workgroups of 16 outputs plus one for the magnetization; EXTERNAL none.
// Arrays are staged in LDS for grids up to BATCH_FORCE_STAGE columns (48 KB,
// and at most 64 VGPRs: two workgroups per compute unit, so that the many
// ring items of a cycle run two at a time on each unit).
constexpr int BATCH_FORCE_STAGE = 2048;
constexpr int BATCH_SHEET_WORDS = ((BATCH_FORCE_STAGE + 63) / 64) * 65;
constexpr int BATCH_FORCE_LDS = BATCH_SHEET_WORDS > 3 * BATCH_FORCE_STAGE ? BATCH_SHEET_WORDS : 3 * BATCH_FORCE_STAGE;

static __global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void kb_force(const GridDesc *__restrict__ gd, const Cycle *__restrict__ cy)
{
    __shared__ double L[BATCH_FORCE_LDS];
    __shared__ double M[2];
    const int n = cy->n;
    const int total = cy->off_force[n];
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int a = find_member(cy->off_force, n, e);
        const GridDesc &g = gd[cy->slot[a]];
        const int li = e - cy->off_force[a];
        __syncthreads();
        if (g.model == 0) {
            if (g.nx <= BATCH_FORCE_STAGE)
                force_hmf_block<true, BATCH_FORCE_STAGE>(g.rho, g.cs, g.sn, g.F, g.nx, g.dx, g.mxmy, g.hist,
                                                         g.hcount, g.hcap, L, M);
            else
                force_hmf_block<false>(g.rho, g.cs, g.sn, g.F, g.nx, g.dx, g.mxmy, g.hist, g.hcount, g.hcap, L, M);
        } else if (g.model == 2) {
            if (g.nx <= BATCH_FORCE_STAGE)
                force_sheet_block<true>(g.rho, g.F, g.nx, g.sheetK, L);
            else
                force_sheet_block<false>(g.rho, g.F, g.nx, g.sheetK, L);
        } else if (g.model == 1) {
            const int nb = (g.nx + 15) / 16;
            if (li < nb) {
                const int i = li * 16 + (threadIdx.x >> 6);
                if (i < g.nx) force_ring_output(g.rho, g.K, g.F, g.nx, g.dx, i);
            } else if (g.nx <= BATCH_FORCE_STAGE) {
                magnetization_block<true, BATCH_FORCE_STAGE>(g.rho, g.cs, g.sn, g.nx, g.dx, g.mxmy, g.hist, g.hcount,
                                                             g.hcap, L);
            } else {
                magnetization_block<false>(g.rho, g.cs, g.sn, g.nx, g.dx, g.mxmy, g.hist, g.hcount, g.hcap, L);
            }
        }
    }
}

template <typename T, int R>
static __global__ __launch_bounds__(256) void kb_kick(const GridDesc *__restrict__ gd, const Cycle *__restrict__ cy)
{
    const int n = cy->n;
    const int total = cy->off_kick[n];
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int a = find_member(cy->off_kick, n, e);
        const GridDesc &g = gd[cy->slot[a]];
        const int li = e - cy->off_kick[a];
        const int ntx = (g.nx + 255) / 256;
        const int tx = li % ntx, ty = li / ntx;
        const int kin = cy->kin[a];
        const T *fin = (const T *)g.f[kin];
        T *fout = (T *)g.f[kin ^ 1];
        if (g.bc_p == BC_PERIODIC)
            kick_tile<T, BC_PERIODIC, R>(fin, fout, g.Fkick, g.dt, g.dp, g.nx, g.np, tx, ty);
        else
            kick_tile<T, BC_ZERO, R>(fin, fout, g.Fkick, g.dt, g.dp, g.nx, g.np, tx, ty);
    }
}

// The kick fused with the two half drifts after it (the second of one step,
// the first of the next) for the members whose tables allow it: tiles of 230
// columns by 16 rows with 8 columns of slack, as the single-grid kernel, or,
// for a member whose drift offsets spread more inside a tile (coarse p, fine
// x, long steps), tiles of 182 columns with 56 of slack (the same 256 kicked
// columns and four waves, more kicked columns per output).  Periodic p only.
constexpr int KB_KD_TW = 230;
constexpr int KB_KD_TW_WIDE = 182, KD_SPR_WIDE = 56;
// (five waves per SIMD: the FP64 form fits them without spilling)
template <typename T, int PF>
static __global__ __launch_bounds__(KDGeom<KB_KD_TW>::NT) __attribute__((amdgpu_waves_per_eu(5)))
void kb_kick_drift(const GridDesc *__restrict__ gd, const Cycle *__restrict__ cy)
{
    using G = KDGeom<KB_KD_TW>;
    using GW = KDGeom<KB_KD_TW_WIDE, KD_SPR_WIDE>;
    static_assert(G::NT == GW::NT && G::NW == GW::NW && G::W1 == GW::W1 && G::W2 == GW::W2 && G::KLD == GW::KLD &&
                      G::NBUF == GW::NBUF,
                  "one workgroup shape and wave roles for both tile widths");
    constexpr int MLD = G::MLD > GW::MLD ? G::MLD : GW::MLD;
    __shared__ __attribute__((aligned(16))) T kbuf[G::NBUF * G::KLD];
    __shared__ __attribute__((aligned(16))) T mbuf[G::NBUF * MLD];
    const int n = cy->n;
    const int total = cy->off_kd[n];
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int a = find_member(cy->off_kd, n, e);
        const GridDesc &g = gd[cy->slot[a]];
        const int li = e - cy->off_kd[a];
        const int tw = g.kd_wide ? KB_KD_TW_WIDE : KB_KD_TW;
        const int ntx = (g.nx + tw - 1) / tw;
        const int tx = li % ntx, ty = li / ntx;
        const int kin = cy->kin[a];
        const T *fin = (const T *)g.f[kin];
        T *fout = (T *)g.f[kin ^ 1];
        const bool full = (ty + 1) * ROWS_PER_BLOCK <= g.np && (g.nx & 1) == 0;
        const int rw = G::role(threadIdx.x >> 6, e % G::NW);
        const bool p2 = rw >= G::W1 && rw < G::W1 + G::W2;
        __syncthreads();  // the previous item's LDS rows are consumed
#define KDB(TW, SPR, BX, FL, P)                                                                                     \
    kick_drift_tile<T, BX, BC_PERIODIC, TW, PF, 1, FL, P, SPR>(fin, fout, g.Fkick, g.dt, g.dp, g.dm, g.dw, g.dw,   \
                                                               g.kbase, g.krel, g.part, g.nx, g.np, tx, ty, rw, kbuf, \
                                                               mbuf)
#define KDB2(TW, SPR, BX, FL)     \
    if (p2)                       \
        KDB(TW, SPR, BX, FL, true); \
    else                          \
        KDB(TW, SPR, BX, FL, false)
#define KDB4(TW, SPR)                              \
    if (g.bc_x == BC_PERIODIC) {                   \
        if (full) {                                \
            KDB2(TW, SPR, BC_PERIODIC, true);      \
        } else {                                   \
            KDB2(TW, SPR, BC_PERIODIC, false);     \
        }                                          \
    } else {                                       \
        if (full) {                                \
            KDB2(TW, SPR, BC_ZERO, true);          \
        } else {                                   \
            KDB2(TW, SPR, BC_ZERO, false);         \
        }                                          \
    }
        if (g.kd_wide) {
            KDB4(KB_KD_TW_WIDE, KD_SPR_WIDE)
        } else {
            KDB4(KB_KD_TW, KD_SPR)
        }
#undef KDB4
#undef KDB2
#undef KDB
    }
}

// Streaming copy (bandwidth ceiling): one 16-byte vector per thread, one
// 4 KiB tile per workgroup (the fastest of the copy shapes measured on the
// chip for buffers larger than its last-level cache).
static __global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n)
{
    const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

}  // namespace vk
