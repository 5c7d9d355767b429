// Kernel launchers of the library, one translation unit per kernel family
// (compiled in parallel); declared in vlasov_internal.hpp.
#include "vlasov_internal.hpp"

namespace vlasov_detail {

template <typename T, int TW, int RB>
int launch_kick_drift_t(vlasov_ctx *c, int ta, double h)
{
    // one kicked column per thread (whole wavefronts); the two half drifts
    // run on waves of their own
    constexpr int NT = vk::KDGeom<TW>::NT;
    const vlasov_params &P = c->P;
    const int ntx = (int)((P.nx + TW - 1) / TW), nty = (int)((c->nblk + RB - 1) / RB);
    const dim3 grid((unsigned)vk::xcd_grid(ntx, nty));
    const T *fin = (const T *)c->fcur();
    T *fout = (T *)c->fnext();
    const double *F = force_ptr(c);
    const int tb = (ta + 1) % c->nsub;
    const int32_t *dm2 = c->dm(tb);
    const double4 *dw1 = c->dw(ta), *dw2 = c->dw(tb);
    const int32_t *kbase = c->at<int32_t>(c->L.kd_base) + (size_t)ta * (size_t)c->nblk;
    const int32_t *krel = c->at<int32_t>(c->L.kd_rel) + (size_t)ta * (size_t)P.np;
    double *part = c->at<double>(c->L.part);
    const int nx = (int)P.nx, np = (int)P.np;
#define KD_LAUNCH(BX, BP)                                                                                        \
    launch(c, VLASOV_K_KICK_DRIFT2, vk::k_kick_drift<T, BX, BP, TW, kd_pf<T>(), RB>, grid, dim3(NT), fin, fout, F, \
           h, c->dp, dm2, dw1, dw2, kbase, krel, part, nx, np, ntx, nty)
    if (P.bc_x == VLASOV_BC_PERIODIC) {
        if (P.bc_p == VLASOV_BC_PERIODIC) KD_LAUNCH(vk::BC_PERIODIC, vk::BC_PERIODIC); else KD_LAUNCH(vk::BC_PERIODIC, vk::BC_ZERO);
    } else {
        if (P.bc_p == VLASOV_BC_PERIODIC) KD_LAUNCH(vk::BC_ZERO, vk::BC_PERIODIC); else KD_LAUNCH(vk::BC_ZERO, vk::BC_ZERO);
    }
#undef KD_LAUNCH
    int rc = check_launch("kick+drift");
    if (rc == VLASOV_OK) c->cur ^= 1;
    return rc;
}

template <typename T, int TW>
int launch_kick_drift_w(vlasov_ctx *c, int ta, double h)
{
    switch (c->kd_rb) {
    case 4:
        return launch_kick_drift_t<T, TW, 4>(c, ta, h);
    case 3:
        return launch_kick_drift_t<T, TW, 3>(c, ta, h);
    case 2:
        return launch_kick_drift_t<T, TW, 2>(c, ta, h);
    default:
        return launch_kick_drift_t<T, TW, 1>(c, ta, h);
    }
}

// Kick k (step size h), the filter if `filt`, then the half drift of table k
// and (tb >= 0, then with partial sums) that of table tb = k + 1 mod nsub:
// the fused kernel where the tables allow it and the launch shape asks for

template int launch_kick_drift_w<double, 230>(vlasov_ctx *, int, double);
template int launch_kick_drift_w<double, 486>(vlasov_ctx *, int, double);

}  // namespace vlasov_detail
