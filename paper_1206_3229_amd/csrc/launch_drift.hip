// Kernel launchers of the library, one translation unit per kernel family
// (compiled in parallel); declared in vlasov_internal.hpp.
#include "vlasov_internal.hpp"

namespace vlasov_detail {

template <typename T, int NT>
int launch_drift_nt(vlasov_ctx *c, int ta, int tb, bool partials)
{
    const int npass = tb >= 0 ? 2 : 1;
    const vlasov_params &P = c->P;
    const int tw = vk::DriftShape<NT, DRIFT_V, 0>::TW;  // columns per workgroup
    const int ntx = (int)((P.nx + tw - 1) / tw), nty = (int)c->nblk;
    const dim3 grid((unsigned)vk::xcd_grid(ntx, nty));
    const T *fin = (const T *)c->fcur();
    T *fout = (T *)c->fnext();
    const int32_t *dm1 = c->dm(ta), *dm2 = c->dm(tb >= 0 ? tb : ta);
    const double4 *dw1 = c->dw(ta), *dw2 = c->dw(tb >= 0 ? tb : ta);
    double *part = c->at<double>(c->L.part);
    const int nx = (int)P.nx, np = (int)P.np;
    const int kid = npass == 2 ? VLASOV_K_DRIFT2 : VLASOV_K_DRIFT;
#define DRIFT_LAUNCH(NP, BC, PT)                                                                                      \
    launch(c, kid, vk::k_drift<T, NP, BC, PT, NT, DRIFT_V, 0, DRIFT_PF>, grid, dim3(NT), fin, fout, dm1, dw1, dm2,   \
           dw2, part, nx, np, ntx, nty)
    if (P.bc_x == VLASOV_BC_PERIODIC) {
        if (npass == 2) {
            if (partials) DRIFT_LAUNCH(2, vk::BC_PERIODIC, true); else DRIFT_LAUNCH(2, vk::BC_PERIODIC, false);
        } else {
            if (partials) DRIFT_LAUNCH(1, vk::BC_PERIODIC, true); else DRIFT_LAUNCH(1, vk::BC_PERIODIC, false);
        }
    } else {
        if (npass == 2) {
            if (partials) DRIFT_LAUNCH(2, vk::BC_ZERO, true); else DRIFT_LAUNCH(2, vk::BC_ZERO, false);
        } else {
            if (partials) DRIFT_LAUNCH(1, vk::BC_ZERO, true); else DRIFT_LAUNCH(1, vk::BC_ZERO, false);
        }
    }
#undef DRIFT_LAUNCH
    int rc = check_launch("drift");
    if (rc == VLASOV_OK) c->cur ^= 1;
    return rc;
}

template <typename T>
int launch_drift(vlasov_ctx *c, int ta, int tb, bool partials)
{
    switch (c->tune.drift_threads) {
    case 64:
        return launch_drift_nt<T, 64>(c, ta, tb, partials);
    case 256:
        return launch_drift_nt<T, 256>(c, ta, tb, partials);
    default:
        return launch_drift_nt<T, 128>(c, ta, tb, partials);
    }
}

template int launch_drift<float>(vlasov_ctx *, int, int, bool);
template int launch_drift<double>(vlasov_ctx *, int, int, bool);

}  // namespace vlasov_detail
