// Kernel launchers of the library, one translation unit per kernel family
// (compiled in parallel); declared in vlasov_internal.hpp.
#include "vlasov_internal.hpp"

namespace vlasov_detail {

template <typename T, int KR>
int launch_kick_r(vlasov_ctx *c, double h)
{
    const vlasov_params &P = c->P;
    const int ntx = (int)((P.nx + 255) / 256), nty = (int)((P.np + KR - 1) / KR);
    const dim3 grid((unsigned)vk::xcd_grid(ntx, nty));
    const T *fin = (const T *)c->fcur();
    T *fout = (T *)c->fnext();
    const double *F = force_ptr(c);
    if (P.bc_p == VLASOV_BC_PERIODIC)
        launch(c, VLASOV_K_KICK, vk::k_kick<T, vk::BC_PERIODIC, KR>, grid, dim3(256), fin, fout, F, h, c->dp,
               (int)P.nx, (int)P.np, ntx, nty);
    else
        launch(c, VLASOV_K_KICK, vk::k_kick<T, vk::BC_ZERO, KR>, grid, dim3(256), fin, fout, F, h, c->dp,
               (int)P.nx, (int)P.np, ntx, nty);
    int rc = check_launch("kick");
    if (rc == VLASOV_OK) c->cur ^= 1;
    return rc;
}

template <typename T>
int launch_kick(vlasov_ctx *c, double h)
{
    switch (c->tune.kick_rows) {
    case 8:
        return launch_kick_r<T, 8>(c, h);
    case 16:
        return launch_kick_r<T, 16>(c, h);
    default:
        return launch_kick_r<T, 32>(c, h);
    }
}

// Kick of step size h (w_k dt) with the last force.

template <typename T>
int launch_filter(vlasov_ctx *c)
{
    const vlasov_params &P = c->P;
    const int ntx = (int)((P.nx + 255) / 256), nty = (int)((P.np + FILTER_R - 1) / FILTER_R);
    const dim3 grid((unsigned)vk::xcd_grid(ntx, nty));
    const T *fin = (const T *)c->fcur();
    T *fout = (T *)c->fnext();
    const double cf = P.filter_strength / 256.0;
    if (P.bc_p == VLASOV_BC_PERIODIC)
        launch(c, VLASOV_K_FILTER, vk::k_filter_p<T, vk::BC_PERIODIC, FILTER_R>, grid, dim3(256), fin, fout, cf,
               (int)P.nx, (int)P.np, ntx, nty);
    else
        launch(c, VLASOV_K_FILTER, vk::k_filter_p<T, vk::BC_ZERO, FILTER_R>, grid, dim3(256), fin, fout, cf,
               (int)P.nx, (int)P.np, ntx, nty);
    int rc = check_launch("filter");
    if (rc == VLASOV_OK) c->cur ^= 1;
    return rc;
}


template <typename T>
int launch_kick_filter(vlasov_ctx *c, double h)
{
    const vlasov_params &P = c->P;
    const int ntx = (int)((P.nx + 255) / 256), nty = (int)((P.np + FILTER_R - 1) / FILTER_R);
    const dim3 grid((unsigned)vk::xcd_grid(ntx, nty));
    const T *fin = (const T *)c->fcur();
    T *fout = (T *)c->fnext();
    const double cf = P.filter_strength / 256.0;
    if (P.bc_p == VLASOV_BC_PERIODIC)
        launch(c, VLASOV_K_FILTER, vk::k_kick_filter<T, vk::BC_PERIODIC, FILTER_R>, grid, dim3(256), fin, fout,
               force_ptr(c), h, c->dp, cf, (int)P.nx, (int)P.np, ntx, nty);
    else
        launch(c, VLASOV_K_FILTER, vk::k_kick_filter<T, vk::BC_ZERO, FILTER_R>, grid, dim3(256), fin, fout,
               force_ptr(c), h, c->dp, cf, (int)P.nx, (int)P.np, ntx, nty);
    int rc = check_launch("kick and filter");
    if (rc == VLASOV_OK) c->cur ^= 1;
    return rc;
}

// The kick followed by the filter: one pass with the local spline, the
// transposed kick and then the filter with the global spline.

// ---------------------------------------------------------------------------
// Global spline (eq. tridiagsys): one workgroup per line; the kick runs on the
// rows of the transpose.
// ---------------------------------------------------------------------------
template <typename T>
int gs_drift_t(vlasov_ctx *c, int table, bool partials)
{
    const vlasov_params &P = c->P;
    const T *fin = (const T *)c->fcur();
    T *fout = (T *)c->fnext();
    const int32_t *dm = c->dm(table);
    const double4 *dw = c->dw(table);
    const double *g = c->at<double>(c->L.gs_g);
    const double *nof = nullptr;
    if (P.bc_x == VLASOV_BC_PERIODIC)
        launch(c, VLASOV_K_DRIFT, vk::k_gs_line<T, vk::BC_PERIODIC, false>, dim3((unsigned)P.np), dim3(vk::GS_NT), fin,
               fout, (int)P.nx, dm, dw, nof, 0.0, 0.0, g);
    else
        launch(c, VLASOV_K_DRIFT, vk::k_gs_line<T, vk::BC_ZERO, false>, dim3((unsigned)P.np), dim3(vk::GS_NT), fin,
               fout, (int)P.nx, dm, dw, nof, 0.0, 0.0, g);
    int rc = check_launch("global-spline drift");
    if (rc) return rc;
    c->cur ^= 1;
    if (partials) {
        launch(c, VLASOV_K_DRIFT, vk::k_partials<T>, dim3((unsigned)((P.nx + 255) / 256), (unsigned)c->nblk),
               dim3(256), (const T *)c->fcur(), c->at<double>(c->L.part), (int)P.nx, (int)P.np);
        rc = check_launch("partial sums");
    }
    return rc;
}

template <typename T>
int gs_kick_t(vlasov_ctx *c, double h)
{
    const vlasov_params &P = c->P;
    const int nx = (int)P.nx, np = (int)P.np;
    T *A = (T *)c->fcur(), *B = (T *)c->fnext();
    const unsigned t1 = (unsigned)(((nx + 63) / 64) * ((np + 63) / 64));
    launch(c, VLASOV_K_KICK, vk::k_transpose<T>, dim3(t1), dim3(256), (const T *)A, B, np, nx);  // B = A^T
    const int32_t *nodm = nullptr;
    const double4 *nodw = nullptr;
    const double *g = c->at<double>(c->L.gs_g);
    if (P.bc_p == VLASOV_BC_PERIODIC)
        launch(c, VLASOV_K_KICK, vk::k_gs_line<T, vk::BC_PERIODIC, true>, dim3((unsigned)nx), dim3(vk::GS_NT),
               (const T *)B, A, np, nodm, nodw, force_ptr(c), h, c->dp, g);
    else
        launch(c, VLASOV_K_KICK, vk::k_gs_line<T, vk::BC_ZERO, true>, dim3((unsigned)nx), dim3(vk::GS_NT),
               (const T *)B, A, np, nodm, nodw, force_ptr(c), h, c->dp, g);
    launch(c, VLASOV_K_KICK, vk::k_transpose<T>, dim3(t1), dim3(256), (const T *)A, B, nx, np);  // B = A^T
    int rc = check_launch("global-spline kick");
    if (rc == VLASOV_OK) c->cur ^= 1;
    return rc;
}


template int launch_kick<float>(vlasov_ctx *, double);
template int launch_kick<double>(vlasov_ctx *, double);
template int launch_filter<float>(vlasov_ctx *);
template int launch_filter<double>(vlasov_ctx *);
template int launch_kick_filter<float>(vlasov_ctx *, double);
template int launch_kick_filter<double>(vlasov_ctx *, double);
template int gs_drift_t<float>(vlasov_ctx *, int, bool);
template int gs_drift_t<double>(vlasov_ctx *, int, bool);
template int gs_kick_t<float>(vlasov_ctx *, double);
template int gs_kick_t<double>(vlasov_ctx *, double);

}  // namespace vlasov_detail
