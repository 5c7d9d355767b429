/*
 * Plain CPU oracle of the time-split semi-Lagrangian Vlasov solver of
 * T. M. Rocha Filho, "Solving the Vlasov equation for one-dimensional models
 * with long range interactions on a GPU" (arXiv:1206.3229).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU solver is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * solver library neither links nor includes anything from here, and this
 * file includes nothing from the solver.
 *
 * Arithmetic is IEEE FP64 throughout (the paper computes in double precision,
 * Sec. 4).  A second storage mode keeps f in FP32 between sweeps and runs the
 * stencil and spline in FP32 while every reduction and the force stay FP64.
 * The file must be compiled with -ffp-contract=off: products and sums are
 * rounded exactly where written, and fused multiply-adds appear only as
 * explicit fma()/fmaf() calls.
 *
 * Threads (OpenMP, compiled with -fopenmp): the work is split over whole
 * lines only (rows of a drift, columns of a kick, a density, a filter or a
 * moment, outputs of the ring convolution).  Every line is computed by one
 * thread exactly as the serial loop would, and sums that run over lines are
 * accumulated afterwards in line order, so results do not depend on the
 * number of threads.
 *
 * Where the paper is silent the following readings are used (each one is
 * restated where it is applied):
 *   R1  the second difference of eq. (findif) carries no 1/du^2; the spline
 *       coefficients of eq. (splinecoeffs) carry du^2, so the two cancel and
 *       the unscaled stencil sum D is combined with (alpha^3-alpha)/6 directly;
 *   R2  n nodes per axis, u_i = umin + i*du, du = (umax-umin)/n;
 *   R3  per-axis boundary: periodic, or zero extension (every sample outside
 *       [0, n) of the line reads 0);
 *   R4  the foot of node i lies at i + xi cells, xi = -(v*tau)/h; m = floor(xi),
 *       theta = xi - m, and a rounded theta of 1 becomes 0 with m+1;
 *   R5  force integrals by the rectangle rule on the grid;
 *   R6  fixed association of every sum (needed for run-to-run and
 *       implementation-independent bit patterns): see sum64 below;
 *   R7  the mean-field potentials are normalised to unit total mass;
 *   R8  sines, cosines and square roots of the node tables (eqs. mxmydef,
 *       hmfmeanforce, ringpot) are the C library's sin, cos and sqrt of each
 *       argument, each called on its own.  The file must therefore also be
 *       compiled with -fno-builtin-sin -fno-builtin-cos -fno-builtin-sincos:
 *       gcc otherwise merges a sin and a cos of one argument into a sincos
 *       call, whose result can differ in the last bit where the exact value
 *       lies almost half-way between two doubles;
 *   R9  entropy -int f log f over the points where f > 0 (the spline can
 *       make f slightly negative; that mass is reported on its own);
 *   R10 the global spline of eq. (tridiagsys) with the diagonal read as
 *       2 f''_i/3 (the standard spline condition of the cited method; as
 *       printed, f''_i/3, the periodic system is singular at the shortest
 *       wave), periodic or continued by zeros like the samples (R3);
 *   R11 higher-order time splitting (named in the conclusions as an
 *       extension, after Arber and Vann): a step of size dt is the
 *       composition of the Sec. 3 step (half drift, force, kick, half drift)
 *       with sizes w_k dt; weights of the fourth-order symmetric compositions
 *       of Yoshida / Forest-Ruth (w1, w0, w1) and Suzuki (p, p, 1-4p, p, p);
 *       the drifts of consecutive substeps stay separate sweeps, as those of
 *       consecutive steps do;
 *   R12 filtering (the same passage): after the last kick of every k-th step,
 *       f <- f - (sigma/256) delta_p^8 f along each column (delta_p^8 the
 *       eighth central difference, binomial weights), which damps the mode
 *       of wavenumber kappa by the factor 1 - sigma sin^8(kappa/2) and keeps
 *       every p-moment of degree below 8 of each column.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { MODEL_HMF = 0, MODEL_RING = 1, MODEL_SHEET = 2, MODEL_EXTERNAL = 3 };
enum { BC_PERIODIC = 0, BC_ZERO = 1 };
enum { STORE_F64 = 0, STORE_F32 = 1 };

enum { SPLINE_FD = 0, SPLINE_GS = 1 };
enum { SPLIT_STRANG = 0, SPLIT_TRIPLE_JUMP = 1, SPLIT_SUZUKI = 2 };

typedef struct {
    int32_t model, storage, bc_x, bc_p;
    int32_t spline;       /* SPLINE_FD: f'' by eq. (findif); SPLINE_GS: by eq. (tridiagsys) */
    int32_t splitting;    /* R11 */
    int32_t filter_every; /* R12: 0 = no filter */
    int32_t pad;
    int64_t nx, np;
    double xmin, xmax, pmin, pmax, dt, ring_eps, sheet_G;
    double filter_strength; /* R12: sigma */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* Eq. (findif): eighth-order centred second difference.  Coefficients are  */
/* the correctly rounded doubles of the printed rationals.                  */
/* ------------------------------------------------------------------------ */
static const double FD0 = -205.0 / 72.0;
static const double FD1 = 8.0 / 5.0;
static const double FD2 = -1.0 / 5.0;
static const double FD3 = 8.0 / 315.0;
static const double FD4 = -1.0 / 560.0;

/* R3: one sample of a line of n values spaced by `stride`. */
static double sample(const double *line, int64_t n, int64_t stride, int64_t k, int bc)
{
    if (bc == BC_PERIODIC) {
        k %= n;
        if (k < 0) k += n;
        return line[k * stride];
    }
    return (k >= 0 && k < n) ? line[k * stride] : 0.0;
}

/* Eq. (findif) at node l, without the 1/du^2 (R1).  The symmetric pairs are
 * added first and accumulated from the outermost pair inwards. */
static double second_difference(const double *line, int64_t n, int64_t stride, int64_t l, int bc)
{
#define S(o) sample(line, n, stride, l + (o), bc)
    double s = FD4 * (S(-4) + S(4));
    s = fma(FD3, S(-3) + S(3), s);
    s = fma(FD2, S(-2) + S(2), s);
    s = fma(FD1, S(-1) + S(1), s);
    return fma(FD0, S(0), s);
#undef S
}

static float samplef(const double *line, int64_t n, int64_t stride, int64_t k, int bc)
{
    return (float)sample(line, n, stride, k, bc);
}

static float second_difference_f32(const double *line, int64_t n, int64_t stride, int64_t l, int bc)
{
#define S(o) samplef(line, n, stride, l + (o), bc)
    float s = (float)FD4 * (S(-4) + S(4));
    s = fmaf((float)FD3, S(-3) + S(3), s);
    s = fmaf((float)FD2, S(-2) + S(2), s);
    s = fmaf((float)FD1, S(-1) + S(1), s);
    return fmaf((float)FD0, S(0), s);
#undef S
}

/* ------------------------------------------------------------------------ */
/* Eqs. (splinegen), (splinecoeffs): foot cell and spline weights.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t m;
    double alpha, beta, gamma, delta; /* gamma, delta without du^2 (R1) */
} foot_t;

/* R4.  A non-finite or absurdly large shift yields NaN weights (and m = 0), so
 * a blown-up force poisons the line instead of indexing out of range. */
static foot_t foot_of_shift(double a)
{
    foot_t w;
    double xi = -a;
    if (!(fabs(xi) < 2147483648.0)) {
        w.m = 0;
        w.alpha = w.beta = w.gamma = w.delta = NAN;
        return w;
    }
    double fl = floor(xi);
    double th = xi - fl;
    w.m = (int64_t)fl;
    if (th >= 1.0) {
        th = 0.0;
        w.m += 1;
    }
    w.alpha = 1.0 - th;
    w.beta = th;
    w.gamma = ((w.alpha * w.alpha) * w.alpha - w.alpha) / 6.0;
    w.delta = ((w.beta * w.beta) * w.beta - w.beta) / 6.0;
    return w;
}

/* Backward semi-Lagrangian update of one line (Sec. 3): the new value at node
 * i is the cubic spline of the old line evaluated at the foot i + xi, i.e.
 * eq. (splinegen) on the cell [k, k+1], k = i + m, with f'' from eq. (findif).
 * The four terms are accumulated in the order gamma, delta, beta, alpha. */
static void interpolate_line(const double *in, double *out, int64_t n, int64_t stride, double shift,
                             int bc, int storage)
{
    foot_t w = foot_of_shift(shift);
    if (storage == STORE_F32) {
        float al = (float)w.alpha, be = (float)w.beta, ga = (float)w.gamma, de = (float)w.delta;
        for (int64_t i = 0; i < n; i++) {
            int64_t k = i + w.m;
            float Dk = second_difference_f32(in, n, stride, k, bc);
            float Dk1 = second_difference_f32(in, n, stride, k + 1, bc);
            float r = ga * Dk;
            r = fmaf(de, Dk1, r);
            r = fmaf(be, samplef(in, n, stride, k + 1, bc), r);
            out[i * stride] = (double)fmaf(al, samplef(in, n, stride, k, bc), r);
        }
        return;
    }
    for (int64_t i = 0; i < n; i++) {
        int64_t k = i + w.m;
        double Dk = second_difference(in, n, stride, k, bc);
        double Dk1 = second_difference(in, n, stride, k + 1, bc);
        double r = w.gamma * Dk;
        r = fma(w.delta, Dk1, r);
        r = fma(w.beta, sample(in, n, stride, k + 1, bc), r);
        out[i * stride] = fma(w.alpha, sample(in, n, stride, k, bc), r);
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. (tridiagsys): the global spline.  Continuity of the first derivative  */
/* across the nodes gives, for D_i = f''_i du^2 (R1) and reading the printed */
/* diagonal f''_i/3 as 2 f''_i/3 (R10), the tridiagonal system               */
/*   D_{i-1} + 4 D_i + D_{i+1} = 6 (f_{i+1} - 2 f_i + f_{i-1}).              */
/* Periodic lines: the cyclic system, solved by Thomas elimination with the  */
/* Sherman-Morrison correction for the two corner entries.  Zero extension:  */
/* the line continued by zeros on both sides (GS_PAD cells, beyond which D   */
/* is below 0.27^GS_PAD of its size and set to 0), solved by Thomas.         */
/* ------------------------------------------------------------------------ */
#define GS_PAD 64

/* Solves the (1, 4, 1) system with diagonal b[] (b[0] and b[n-1] may be
 * modified by the caller) for right-hand side r[] into x[]; work w[n]. */
static void thomas_141(const double *b, const double *r, double *x, double *w, int64_t n)
{
    double piv = b[0];
    x[0] = r[0] / piv;
    for (int64_t i = 1; i < n; i++) {
        w[i] = 1.0 / piv;
        piv = b[i] - w[i];
        x[i] = (r[i] - x[i - 1]) / piv;
    }
    for (int64_t i = n - 2; i >= 0; i--) x[i] -= w[i + 1] * x[i + 1];
}

/* D of a line of n samples (spacing `stride`).  Periodic: D[0..n).  Zero
 * extension: D[0..n + 2 GS_PAD), D[k + GS_PAD] for node k in [-GS_PAD, n + GS_PAD). */
static void gs_second_derivatives(const double *line, int64_t n, int64_t stride, int bc, double *D)
{
    if (bc == BC_PERIODIC) {
        double *b = malloc((size_t)n * sizeof(double)), *r = malloc((size_t)n * sizeof(double));
        double *u = malloc((size_t)n * sizeof(double)), *z = malloc((size_t)n * sizeof(double));
        double *w = malloc((size_t)n * sizeof(double));
        for (int64_t i = 0; i < n; i++) {
            const double fm = line[((i - 1 + n) % n) * stride], f0 = line[i * stride], fp = line[((i + 1) % n) * stride];
            r[i] = 6.0 * ((fp - 2.0 * f0) + fm);
            b[i] = 4.0;
            u[i] = 0.0;
        }
        /* A = A' + u v^T with u = (g, 0, .., 0, 1), v = (1, 0, .., 0, 1/g), g = -4 */
        const double g = -4.0;
        b[0] -= g;
        b[n - 1] -= 1.0 / g;
        u[0] = g;
        u[n - 1] = 1.0;
        thomas_141(b, r, D, w, n);
        thomas_141(b, u, z, w, n);
        const double fac = (D[0] + D[n - 1] / g) / ((1.0 + z[0]) + z[n - 1] / g);
        for (int64_t i = 0; i < n; i++) D[i] -= fac * z[i];
        free(b);
        free(r);
        free(u);
        free(z);
        free(w);
        return;
    }
    const int64_t N = n + 2 * GS_PAD;
    double *b = malloc((size_t)N * sizeof(double)), *r = malloc((size_t)N * sizeof(double));
    double *w = malloc((size_t)N * sizeof(double));
    for (int64_t e = 0; e < N; e++) {
        const int64_t i = e - GS_PAD;
        const double fm = (i - 1 >= 0 && i - 1 < n) ? line[(i - 1) * stride] : 0.0;
        const double f0 = (i >= 0 && i < n) ? line[i * stride] : 0.0;
        const double fp = (i + 1 >= 0 && i + 1 < n) ? line[(i + 1) * stride] : 0.0;
        r[e] = 6.0 * ((fp - 2.0 * f0) + fm);
        b[e] = 4.0;
    }
    thomas_141(b, r, D, w, N);
    free(b);
    free(r);
    free(w);
}

/* The backward semi-Lagrangian update of one line with the global spline:
 * as interpolate_line, with D from eq. (tridiagsys).  FP32 storage: D is
 * solved in FP64 from the stored samples and rounded, the combination runs
 * in FP32. */
static void interpolate_line_gs(const double *in, double *out, int64_t n, int64_t stride, double shift, int bc,
                                int storage)
{
    foot_t w = foot_of_shift(shift);
    double *D = malloc((size_t)(n + 2 * GS_PAD) * sizeof(double));
    gs_second_derivatives(in, n, stride, bc, D);
    for (int64_t i = 0; i < n; i++) {
        int64_t k = i + w.m;
        double Dk, Dk1;
        if (bc == BC_PERIODIC) {
            int64_t q = ((k % n) + n) % n, q1 = (((k + 1) % n) + n) % n;
            Dk = D[q];
            Dk1 = D[q1];
        } else {
            Dk = (k >= -GS_PAD && k < n + GS_PAD) ? D[k + GS_PAD] : 0.0;
            Dk1 = (k + 1 >= -GS_PAD && k + 1 < n + GS_PAD) ? D[k + 1 + GS_PAD] : 0.0;
        }
        if (storage == STORE_F32) {
            float r = (float)w.gamma * (float)Dk;
            r = fmaf((float)w.delta, (float)Dk1, r);
            r = fmaf((float)w.beta, samplef(in, n, stride, k + 1, bc), r);
            out[i * stride] = (double)fmaf((float)w.alpha, samplef(in, n, stride, k, bc), r);
        } else {
            double r = w.gamma * Dk;
            r = fma(w.delta, Dk1, r);
            r = fma(w.beta, sample(in, n, stride, k + 1, bc), r);
            out[i * stride] = fma(w.alpha, sample(in, n, stride, k, bc), r);
        }
    }
    free(D);
}

static void interpolate(const oracle_params *P, const double *in, double *out, int64_t n, int64_t stride,
                        double shift, int bc)
{
    if (P->spline == SPLINE_GS)
        interpolate_line_gs(in, out, n, stride, shift, bc, P->storage);
    else
        interpolate_line(in, out, n, stride, shift, bc, P->storage);
}

static double grid_dx(const oracle_params *P) { return (P->xmax - P->xmin) / (double)P->nx; }
static double grid_dp(const oracle_params *P) { return (P->pmax - P->pmin) / (double)P->np; }
static double node_x(const oracle_params *P, int64_t i) { return P->xmin + (double)i * grid_dx(P); }
static double node_p(const oracle_params *P, int64_t j) { return P->pmin + (double)j * grid_dp(P); }

/* Steps 1 and 4 of Sec. 3 (eqs. step1, step4): advection along x for a time
 * tau at constant momentum; row j moves by p_j*tau/dx cells. */
void oracle_advect_x(const oracle_params *P, const double *f, double *out, double tau)
{
    double dx = grid_dx(P);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < P->np; j++) {
        double shift = (node_p(P, j) * tau) / dx;
        interpolate(P, f + j * P->nx, out + j * P->nx, P->nx, 1, shift, P->bc_x);
    }
}

/* Step 3 of Sec. 3 (eq. step3): advection along p for a time dt with the
 * force of column i; column i moves by F_i*dt/dp cells. */
void oracle_advect_p(const oracle_params *P, const double *f, double *out, const double *F, double dt)
{
    double dp = grid_dp(P);
    const int64_t nx = P->nx, np = P->np;
#pragma omp parallel
    {
        /* each column is copied to a contiguous line, moved, and copied back */
        double *line = malloc((size_t)np * sizeof(double)), *moved = malloc((size_t)np * sizeof(double));
#pragma omp for schedule(static, 64)
        for (int64_t i = 0; i < nx; i++) {
            double shift = (F[i] * dt) / dp;
            for (int64_t j = 0; j < np; j++) line[j] = f[j * nx + i];
            interpolate(P, line, moved, np, 1, shift, P->bc_p);
            for (int64_t j = 0; j < np; j++) out[j * nx + i] = moved[j];
        }
        free(line);
        free(moved);
    }
}

/* ------------------------------------------------------------------------ */
/* R6: association of sums.  A sum over t = 0..n-1 keeps 64 running partial */
/* sums, term t going to partial t mod 64 in ascending t, then combines the */
/* partials pairwise: partial l += partial l+d for d = 32, 16, 8, 4, 2, 1.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double acc[64];
} sum64;

static void sum64_init(sum64 *s) { memset(s, 0, sizeof *s); }
static void sum64_add(sum64 *s, int64_t t, double v) { s->acc[t & 63] = s->acc[t & 63] + v; }
static void sum64_fma(sum64 *s, int64_t t, double a, double b) { s->acc[t & 63] = fma(a, b, s->acc[t & 63]); }
static double sum64_total(sum64 *s)
{
    for (int d = 32; d >= 1; d >>= 1)
        for (int l = 0; l < d; l++) s->acc[l] = s->acc[l] + s->acc[l + d];
    return s->acc[0];
}

/* Column sums over the momentum rows, R6 refined for the 2D sum: rows are
 * taken in blocks of 16 consecutive rows, each block summed serially from 0,
 * and the block sums are combined by sum64 over the block index.  The term of
 * row j is w_j * f (fused) when a weight row is given, else by `term`:
 * TERM_F f, TERM_SQUARE f*f (fused), TERM_FLOGF f*log(f) for f > 0 and 0
 * otherwise (entropy density, R9), TERM_NEG f for f < 0 and 0 otherwise. */
enum { TERM_F = 0, TERM_SQUARE = 1, TERM_FLOGF = 2, TERM_NEG = 3 };

static double column_sum(const oracle_params *P, const double *f, int64_t i, const double *w, int term)
{
    sum64 s;
    sum64_init(&s);
    for (int64_t b = 0; b * 16 < P->np; b++) {
        double blk = 0.0;
        int64_t jend = (b + 1) * 16 < P->np ? (b + 1) * 16 : P->np;
        for (int64_t j = b * 16; j < jend; j++) {
            double v = f[j * P->nx + i];
            if (w)
                blk = fma(w[j], v, blk);
            else if (term == TERM_SQUARE)
                blk = fma(v, v, blk);
            else if (term == TERM_FLOGF)
                blk = blk + (v > 0.0 ? v * log(v) : 0.0);
            else if (term == TERM_NEG)
                blk = blk + (v < 0.0 ? v : 0.0);
            else
                blk = blk + v;
        }
        sum64_add(&s, b, blk);
    }
    return sum64_total(&s);
}

/* Spatial density rho(x_i) = int f dp, rectangle rule (R5). */
void oracle_density(const oracle_params *P, const double *f, double *rho)
{
    double dp = grid_dp(P);
#pragma omp parallel for schedule(static, 64)
    for (int64_t i = 0; i < P->nx; i++) rho[i] = dp * column_sum(P, f, i, NULL, TERM_F);
}

/* Magnetization, eq. (mxmydef): M_x = int cos(theta) rho, M_y = int sin(theta) rho. */
static void magnetization(const oracle_params *P, const double *rho, double *mx, double *my)
{
    double dx = grid_dx(P);
    sum64 c, s;
    sum64_init(&c);
    sum64_init(&s);
    for (int64_t i = 0; i < P->nx; i++) {
        double th = node_x(P, i);
        sum64_fma(&c, i, cos(th), rho[i]);
        sum64_fma(&s, i, sin(th), rho[i]);
    }
    *mx = dx * sum64_total(&c);
    *my = dx * sum64_total(&s);
}

/* Ring model, eq. (ringpot): V(d) = -1/sqrt(2(1+eps-cos d)).  dV/dd =
 * sin d / (2(1+eps-cos d))^{3/2}, written q = 2(1+eps-cos d), sin d/(q sqrt q).
 * The tabulated derivative at separation s cells is made exactly odd
 * (K_{n-s} = -K_s, zero at s = 0 and s = n/2) and the potential exactly even,
 * as the continuous functions are. */
static double ring_dV(double d, double eps)
{
    double q = 2.0 * ((1.0 + eps) - cos(d));
    return sin(d) / (q * sqrt(q));
}

static double ring_V(double d, double eps)
{
    double q = 2.0 * ((1.0 + eps) - cos(d));
    return -1.0 / sqrt(q);
}

static double ring_dV_table(const oracle_params *P, int64_t s)
{
    int64_t n = P->nx;
    double dx = grid_dx(P);
    if (s == 0 || 2 * s == n) return 0.0;
    if (2 * s < n) return ring_dV((double)s * dx, P->ring_eps);
    return -ring_dV((double)(n - s) * dx, P->ring_eps);
}

static double ring_V_table(const oracle_params *P, int64_t s)
{
    int64_t n = P->nx;
    double dx = grid_dx(P);
    if (2 * s > n) s = n - s;
    return ring_V((double)s * dx, P->ring_eps);
}

/* Step 2 of Sec. 3 (eq. step2): mean-field force from the density, for each
 * model, by eq. (meanforce) discretised with the rectangle rule (R5).
 * Writes F[0..nx) and, for the angular models, the magnetization (mx, my). */
void oracle_force(const oracle_params *P, const double *rho, const double *F_ext, double *F, double *mxmy)
{
    int64_t n = P->nx;
    double dx = grid_dx(P);
    double mx = 0.0, my = 0.0;
    if (P->model == MODEL_HMF || P->model == MODEL_RING) magnetization(P, rho, &mx, &my);
    if (mxmy) {
        mxmy[0] = mx;
        mxmy[1] = my;
    }
    if (P->model == MODEL_HMF) {
        /* eq. (hmfmeanforce): F = -sin(theta) M_x + cos(theta) M_y */
        for (int64_t i = 0; i < n; i++) {
            double th = node_x(P, i);
            F[i] = fma(my, cos(th), -(mx * sin(th)));
        }
    } else if (P->model == MODEL_RING) {
        /* F_i = -dx sum_k V'(x_i - x_k) rho_k, direct periodic convolution */
#pragma omp parallel for schedule(static, 16)
        for (int64_t i = 0; i < n; i++) {
            sum64 s;
            sum64_init(&s);
            for (int64_t k = 0; k < n; k++) {
                int64_t d = (i - k) % n;
                if (d < 0) d += n;
                sum64_fma(&s, k, ring_dV_table(P, d), rho[k]);
            }
            F[i] = -(dx * sum64_total(&s));
        }
    } else if (P->model == MODEL_SHEET) {
        /* V = 2 pi G |x|: F_i = 2 pi G (M(>x_i) - M(<x_i)), the cell itself
         * exerting no force.  M(<x_i) = dx P_i with P_i the exclusive prefix
         * sum of rho, M(>x_i) = dx (S - P_i - rho_i).  R6 for the scan: 64
         * contiguous chunks of c = ceil(n/64) cells, a serial exclusive prefix
         * inside each chunk, an inclusive scan of the chunk totals with
         * T_l += T_{l-d} for d = 1, 2, 4, 8, 16, 32, and P_i = (exclusive chunk
         * offset) + (prefix inside the chunk). */
        int64_t c = (n + 63) / 64;
        double tot[64], excl[64];
        for (int l = 0; l < 64; l++) {
            double acc = 0.0;
            for (int64_t i = l * c; i < (l + 1) * c && i < n; i++) acc = acc + rho[i];
            tot[l] = acc;
        }
        for (int d = 1; d < 64; d <<= 1) {
            double nxt[64];
            for (int l = 0; l < 64; l++) nxt[l] = (l >= d) ? tot[l - d] + tot[l] : tot[l];
            memcpy(tot, nxt, sizeof tot);
        }
        for (int l = 0; l < 64; l++) excl[l] = (l == 0) ? 0.0 : tot[l - 1];
        double S = tot[63];
        double K = ((2.0 * M_PI) * P->sheet_G) * dx;
        for (int l = 0; l < 64; l++) {
            double acc = 0.0;
            for (int64_t i = l * c; i < (l + 1) * c && i < n; i++) {
                double Pi = excl[l] + acc;
                F[i] = K * (fma(-2.0, Pi, S) - rho[i]);
                acc = acc + rho[i];
            }
        }
    } else {
        for (int64_t i = 0; i < n; i++) F[i] = F_ext ? F_ext[i] : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* R12: the filter along p.  For each column, with the samples of R3:        */
/*   s_j = sum_m b_m f_{j+m},  b = (1, -8, 28, -56, 70, -56, 28, -8, 1),     */
/* pairs added first and accumulated from the outermost pair inwards like    */
/* the stencil of eq. (findif); out_j = f_j - (sigma/256) s_j as one fma.    */
/* ------------------------------------------------------------------------ */
void oracle_filter_p(const oracle_params *P, const double *f, double *out)
{
    const double c = P->filter_strength / 256.0;
#pragma omp parallel for schedule(static, 64)
    for (int64_t i = 0; i < P->nx; i++) {
        const double *col = f + i;
        for (int64_t j = 0; j < P->np; j++) {
            double v;
            if (P->storage == STORE_F32) {
                float s = samplef(col, P->np, P->nx, j - 4, P->bc_p) + samplef(col, P->np, P->nx, j + 4, P->bc_p);
                s = fmaf(-8.0f, samplef(col, P->np, P->nx, j - 3, P->bc_p) + samplef(col, P->np, P->nx, j + 3, P->bc_p), s);
                s = fmaf(28.0f, samplef(col, P->np, P->nx, j - 2, P->bc_p) + samplef(col, P->np, P->nx, j + 2, P->bc_p), s);
                s = fmaf(-56.0f, samplef(col, P->np, P->nx, j - 1, P->bc_p) + samplef(col, P->np, P->nx, j + 1, P->bc_p), s);
                const float fj = samplef(col, P->np, P->nx, j, P->bc_p);
                s = fmaf(70.0f, fj, s);
                v = (double)fmaf(-(float)c, s, fj);
            } else {
                double s = sample(col, P->np, P->nx, j - 4, P->bc_p) + sample(col, P->np, P->nx, j + 4, P->bc_p);
                s = fma(-8.0, sample(col, P->np, P->nx, j - 3, P->bc_p) + sample(col, P->np, P->nx, j + 3, P->bc_p), s);
                s = fma(28.0, sample(col, P->np, P->nx, j - 2, P->bc_p) + sample(col, P->np, P->nx, j + 2, P->bc_p), s);
                s = fma(-56.0, sample(col, P->np, P->nx, j - 1, P->bc_p) + sample(col, P->np, P->nx, j + 1, P->bc_p), s);
                const double fj = sample(col, P->np, P->nx, j, P->bc_p);
                s = fma(70.0, fj, s);
                v = fma(-c, s, fj);
            }
            out[j * P->nx + i] = v;
        }
    }
}

/* R11: weights w_k of the composition; returns their number.  The decimal
 * constants are the doubles nearest to the exact values. */
int oracle_split_weights(int scheme, double *w)
{
    switch (scheme) {
    case SPLIT_TRIPLE_JUMP: /* w1 = 1/(2 - 2^(1/3)), w0 = -2^(1/3)/(2 - 2^(1/3)) */
        w[0] = 1.3512071919596575;
        w[1] = -1.7024143839193153;
        w[2] = 1.3512071919596575;
        return 3;
    case SPLIT_SUZUKI: /* p = 1/(4 - 4^(1/3)) four times, 1 - 4p in the middle */
        w[0] = w[1] = w[3] = w[4] = 0.4144907717943757;
        w[2] = -0.657963087177503;
        return 5;
    default:
        w[0] = 1.0;
        return 1;
    }
}

/* Storage rounding of the FP32 mode: f lives in FP32 between sweeps. */
static void store_round(const oracle_params *P, double *f)
{
    if (P->storage != STORE_F32) return;
    int64_t N = P->nx * P->np;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < N; t++) f[t] = (double)(float)f[t];
}

/* One time step: the Sec. 3 step (half drift, force from the drifted f, full
 * kick, half drift) applied with the sizes w_k dt of R11 in turn (one
 * substep of size dt for the paper's scheme), the filter of R12 after the
 * last kick when `filtered`.  f is updated in place; `hist` (may be NULL)
 * receives the magnetization of the drifted f of every force evaluation. */
static int split_step(const oracle_params *P, double *f, double *g, double *rho, double *F, const double *F_ext,
                      double *hist, int filtered)
{
    double w[8];
    const int ns = oracle_split_weights(P->splitting, w);
    for (int k = 0; k < ns; k++) {
        const double h = w[k] * P->dt;
        const double tau = 0.5 * h;
        oracle_advect_x(P, f, g, tau);                         /* eq. (step1) */
        oracle_density(P, g, rho);
        oracle_force(P, rho, F_ext, F, hist ? hist + 2 * k : NULL); /* eq. (step2) */
        oracle_advect_p(P, g, f, F, h);                        /* eq. (step3) */
        if (filtered && k == ns - 1) {
            oracle_filter_p(P, f, g);                          /* R12 */
            memcpy(f, g, (size_t)(P->nx * P->np) * sizeof(double));
        }
        oracle_advect_x(P, f, g, tau);                         /* eq. (step4) */
        memcpy(f, g, (size_t)(P->nx * P->np) * sizeof(double));
    }
    return 0;
}

/* Run nsteps time steps in place.  hist (nullable) gets 2 values per force
 * evaluation: 2 * nsteps * (number of substeps).  Step s (from 0) is filtered
 * when filter_every > 0 and s + 1 is a multiple of it. */
int oracle_run(const oracle_params *P, double *f, int64_t nsteps, const double *F_ext, double *hist)
{
    int64_t N = P->nx * P->np;
    double *g = malloc((size_t)N * sizeof(double));
    double *rho = malloc((size_t)P->nx * sizeof(double));
    double *F = malloc((size_t)P->nx * sizeof(double));
    if (!g || !rho || !F) {
        free(g);
        free(rho);
        free(F);
        return -2;
    }
    double w[8];
    const int ns = oracle_split_weights(P->splitting, w);
    store_round(P, f);
    for (int64_t s = 0; s < nsteps; s++) {
        const int filtered = P->filter_every > 0 && (s + 1) % P->filter_every == 0;
        split_step(P, f, g, rho, F, F_ext, hist ? hist + 2 * ns * s : NULL, filtered);
    }
    free(g);
    free(rho);
    free(F);
    return 0;
}

/* Single sweeps in the storage precision (for sweep-level comparisons). */
void oracle_sweep_x(const oracle_params *P, const double *f, double *out, double tau)
{
    oracle_advect_x(P, f, out, tau);
}

void oracle_sweep_p(const oracle_params *P, const double *f, double *out, const double *F, double dt)
{
    oracle_advect_p(P, f, out, F, dt);
}

/* Diagnostics of the current f (the quantities of the accuracy study of
 * Sec. 4.1): out = {mass, momentum, kinetic, potential, energy, M_x, M_y,
 * sum f^2 dx dp, entropy (R9; eq. casimirs with s(f) = -f log f),
 * negative mass dx dp sum_{f<0} f}.  Potential energies with unit-mass normalisation (R7):
 *   HMF   W = (mass^2 - M_x^2 - M_y^2)/2            (eqs. hmfpot, mxmydef)
 *   ring  W = 1/2 dx^2 sum_i sum_k V(x_i-x_k) rho_i rho_k, self term included
 *   sheet W = pi G dx^2 sum_i sum_k |x_i-x_k| rho_i rho_k
 *   external: 0. */
void oracle_moments(const oracle_params *P, const double *f, double *out)
{
    int64_t nx = P->nx, np = P->np;
    double dx = grid_dx(P), dp = grid_dp(P);
    double *pw = malloc((size_t)np * sizeof(double));
    double *kw = malloc((size_t)np * sizeof(double));
    double *rho = malloc((size_t)nx * sizeof(double));
    for (int64_t j = 0; j < np; j++) {
        pw[j] = node_p(P, j);
        kw[j] = 0.5 * (pw[j] * pw[j]);
    }
    sum64 sm, sj, sk, sq, se, sn;
    sum64_init(&sm);
    sum64_init(&sj);
    sum64_init(&sk);
    sum64_init(&sq);
    sum64_init(&se);
    sum64_init(&sn);
    /* column quantities (one column per thread), then their sums in column order */
    double *col = malloc((size_t)(5 * nx) * sizeof(double));
#pragma omp parallel for schedule(static, 64)
    for (int64_t i = 0; i < nx; i++) {
        rho[i] = dp * column_sum(P, f, i, NULL, TERM_F);
        col[i] = dp * column_sum(P, f, i, pw, TERM_F);
        col[nx + i] = dp * column_sum(P, f, i, kw, TERM_F);
        col[2 * nx + i] = dp * column_sum(P, f, i, NULL, TERM_SQUARE);
        col[3 * nx + i] = dp * column_sum(P, f, i, NULL, TERM_FLOGF);
        col[4 * nx + i] = dp * column_sum(P, f, i, NULL, TERM_NEG);
    }
    for (int64_t i = 0; i < nx; i++) {
        sum64_add(&sm, i, rho[i]);
        sum64_add(&sj, i, col[i]);
        sum64_add(&sk, i, col[nx + i]);
        sum64_add(&sq, i, col[2 * nx + i]);
        sum64_add(&se, i, col[3 * nx + i]);
        sum64_add(&sn, i, col[4 * nx + i]);
    }
    free(col);
    double mass = dx * sum64_total(&sm);
    double mom = dx * sum64_total(&sj);
    double kin = dx * sum64_total(&sk);
    double l2 = dx * sum64_total(&sq);
    double entropy = -(dx * sum64_total(&se));
    double negmass = dx * sum64_total(&sn);
    double mx = 0.0, my = 0.0, W = 0.0;
    if (P->model == MODEL_HMF || P->model == MODEL_RING) magnetization(P, rho, &mx, &my);
    if (P->model == MODEL_HMF) {
        W = 0.5 * ((mass * mass - mx * mx) - my * my);
    } else if (P->model == MODEL_RING || P->model == MODEL_SHEET) {
        /* phi_i = sum_k V(x_i - x_k) rho_k (one output per thread), then
         * sum_i phi_i rho_i in order */
        double *phi = malloc((size_t)nx * sizeof(double));
#pragma omp parallel for schedule(static, 16)
        for (int64_t i = 0; i < nx; i++) {
            sum64 sphi;
            sum64_init(&sphi);
            for (int64_t k = 0; k < nx; k++) {
                int64_t d = (i - k) % nx;
                if (d < 0) d += nx;
                double v = (P->model == MODEL_RING) ? ring_V_table(P, d) : (double)(i > k ? i - k : k - i);
                sum64_fma(&sphi, k, v, rho[k]);
            }
            phi[i] = sum64_total(&sphi);
        }
        sum64 sw;
        sum64_init(&sw);
        for (int64_t i = 0; i < nx; i++) sum64_fma(&sw, i, phi[i], rho[i]);
        free(phi);
        double coef = (P->model == MODEL_RING) ? (0.5 * dx) * dx : (((M_PI * P->sheet_G) * dx) * dx) * dx;
        W = coef * sum64_total(&sw);
    }
    out[0] = mass;
    out[1] = mom;
    out[2] = kin;
    out[3] = W;
    out[4] = kin + W;
    out[5] = mx;
    out[6] = my;
    out[7] = l2;
    out[8] = entropy;
    out[9] = negmass;
    free(pw);
    free(kw);
    free(rho);
}

/* Number of threads of the parallel loops (results do not depend on it). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

/* Exposed pieces for the pin tests. */
double oracle_second_difference(const double *line, int64_t n, int64_t l, int bc)
{
    return second_difference(line, n, 1, l, bc);
}

void oracle_foot(double shift, int64_t *m, double *w4)
{
    foot_t w = foot_of_shift(shift);
    *m = w.m;
    w4[0] = w.alpha;
    w4[1] = w.beta;
    w4[2] = w.gamma;
    w4[3] = w.delta;
}

void oracle_interpolate_line(const double *in, double *out, int64_t n, double shift, int bc, int storage)
{
    interpolate_line(in, out, n, 1, shift, bc, storage);
}

void oracle_interpolate_line_gs(const double *in, double *out, int64_t n, double shift, int bc, int storage)
{
    interpolate_line_gs(in, out, n, 1, shift, bc, storage);
}

double oracle_ring_dV(const oracle_params *P, int64_t s) { return ring_dV_table(P, s); }
double oracle_ring_V(const oracle_params *P, int64_t s) { return ring_V_table(P, s); }
