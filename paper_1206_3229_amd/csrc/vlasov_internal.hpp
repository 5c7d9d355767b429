// Internal declarations shared by the host sources of the library (not part
// of the C ABI): the context, the workspace layout and small helpers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "vlasov.h"
#include "vlasov_kernels.hpp"

namespace vlasov_detail {

// Records the message of a failure for vlasov_last_error() and returns code.
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return ::vlasov_detail::fail(VLASOV_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// drift launch shape: NT threads, runs of V columns, no trim, rows requested PF ahead
constexpr int DRIFT_NT = 128, DRIFT_V = 2, DRIFT_PF = 4;
// kick rows per thread (measured best on 4096^2: 16 for FP64, 32 for FP32)
template <typename T> constexpr int kick_rows() { return sizeof(T) == 8 ? 16 : 32; }
// fused kick and drift: default tile width and blocks (FP64 needs 78 VGPRs
// with 32-row tiles, six waves per SIMD, and 68 with 16-row ones, seven);
// rows requested ahead by the kick
constexpr int KD_TW = 230, KD_RB = 2;
// 32-row tiles where the grid still gives at least this many of them, else
// 16-row tiles (twice the workgroups, to fill the chip)
constexpr int64_t KD_RB_MIN_TILES = 2048;
inline int default_kd_blocks(int64_t nx, int64_t nblk)
{
    return ((nx + KD_TW - 1) / KD_TW) * ((nblk + KD_RB - 1) / KD_RB) >= KD_RB_MIN_TILES ? KD_RB : 1;
}
template <typename T> constexpr int kd_pf() { return 2; }
// rows per thread of the filter along p
constexpr int FILTER_R = 16;
// substeps of a step at most (the splittings of vlasov_splitting)
constexpr int MAX_SUB = 5;

// Sizes w_k of the substeps of one step (in units of dt); returns their number.
int split_weights(int scheme, double *w);

// Workspace layout (byte offsets, each 256-aligned).  The drift tables
// (drift_m, drift_w) hold one table per substep (np rows each), the fused
// kick-drift tables one per pair of consecutive substeps (kd_base nblk
// entries, kd_rel np entries each).
struct Layout {
    size_t drift_m, drift_w, kd_base, kd_rel, part, rho, F, Fext, cs, sn, ringK, ringV, mxmy, hist, hcount, mom_out,
        mom_col, mom_phi, gs_g;
    size_t total;
};

inline int64_t nblocks(int64_t np) { return (np + vk::ROWS_PER_BLOCK - 1) / vk::ROWS_PER_BLOCK; }

Layout layout_of(const vlasov_params &p);

// "" if the parameters are valid, else the reason.
std::string validate(const vlasov_params *p);

// "" if the spec of a generated initial condition is valid, else the reason.
std::string validate_ic(const vlasov_ic *ic);

}  // namespace vlasov_detail

struct vlasov_ctx {
    vlasov_params P;
    hipStream_t stream;
    size_t s;  // bytes per stored value
    char *f[2];
    int cur;
    char *ws;
    vlasov_detail::Layout L;
    double dx, dp;
    int64_t nblk;
    bool have_force;
    vlasov_tuning tune;  // launch shapes of the drift and kick
    // device whose static workspace this context holds (vlasov_init_static), or -1
    int static_dev = -1;
    // HIP graphs of gsteps whole steps (vlasov_set_graph; 0: none), captured on
    // cap_stream the first time they are needed, one per current buffer at the
    // start
    int gsteps = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gcur_end[2] = {0, 0};  // current buffer after a replay
    // host copies kept alive for asynchronous uploads
    std::vector<int32_t> h_dm;
    std::vector<double4> h_dw;
    std::vector<int64_t> h_mfull;  // drift foot offset per row, as the fused tables need it
    std::vector<int32_t> h_kd_base, h_kd_rel;
    // substeps of a step (splitting) and steps taken since init (filter schedule)
    int nsub;
    double wsub[vlasov_detail::MAX_SUB];
    int64_t steps_done;
    // kick k and the two half drifts after it (tables k, k+1 mod nsub) can run
    // fused on tiles of kd_rb blocks (drift shifts of every tile within the
    // kicked halo)
    bool kd_ok[vlasov_detail::MAX_SUB];
    // largest spread of the drift offsets o_j inside one such tile (the
    // batched fused kernel has a wider-slack tile for spreads up to 56)
    int64_t kd_spread[vlasov_detail::MAX_SUB];
    int kd_rb;
    // profiling
    bool prof;
    struct Rec {
        int kid;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double ms[VLASOV_K_COUNT];
    int64_t cnt[VLASOV_K_COUNT];

    template <typename U> U *at(size_t off) const { return reinterpret_cast<U *>(ws + off); }
    // drift table of substep k
    const int32_t *dm(int k) const { return at<int32_t>(L.drift_m) + (size_t)k * (size_t)P.np; }
    const double4 *dw(int k) const { return at<double4>(L.drift_w) + (size_t)k * (size_t)P.np; }
    void *fcur() const { return f[cur]; }
    void *fnext() const { return f[cur ^ 1]; }
};

namespace vlasov_detail {
// Force array read by the kick: the caller's table for the EXTERNAL model.
inline const double *force_ptr(const vlasov_ctx *c)
{
    return c->at<double>(c->P.model == VLASOV_MODEL_EXTERNAL ? c->L.Fext : c->L.F);
}

inline hipEvent_t take_event(vlasov_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launches a kernel on the context's stream.  When profiling is on, the
// launch carries its own start/stop events (recorded by the dispatch itself,
// so no extra packets sit between consecutive kernels).
template <typename... KArgs, typename... Args>
void launch(vlasov_ctx *c, int kid, void (*kernel)(KArgs...), dim3 grid, dim3 block, Args... args)
{
    if (c->prof) {
        hipEvent_t a = take_event(c), b = take_event(c);
        if (a && b) {
            hipExtLaunchKernelGGL(kernel, grid, block, 0, c->stream, a, b, 0, static_cast<KArgs>(args)...);
            c->recs.push_back({kid, a, b});
            return;
        }
    }
    kernel<<<grid, block, 0, c->stream>>>(static_cast<KArgs>(args)...);
}

inline int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VLASOV_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return VLASOV_OK;
}

// Launchers (one translation unit per kernel family).  Each enqueues its
// kernel on the context's stream and, on success, makes the output buffer
// the current f.
// Half drift of table ta, then (tb >= 0) that of table tb, in one pass; with
// partials the density partial sums of the result.
template <typename T> int launch_drift(vlasov_ctx *c, int ta, int tb, bool partials);
// Kick of step size h with the last force.
template <typename T> int launch_kick(vlasov_ctx *c, double h);
// The filter along p; the kick of step size h followed by the filter.
template <typename T> int launch_filter(vlasov_ctx *c);
template <typename T> int launch_kick_filter(vlasov_ctx *c, double h);
// Global spline: half drift of table `table` (and its partial sums); kick.
template <typename T> int gs_drift_t(vlasov_ctx *c, int table, bool partials);
template <typename T> int gs_kick_t(vlasov_ctx *c, double h);
// Kick of substep ta (step size h) fused with the half drifts of tables ta
// and ta + 1 mod nsub, on tiles of TW columns.
template <typename T, int TW> int launch_kick_drift_w(vlasov_ctx *c, int ta, double h);
}  // namespace vlasov_detail

