// One Adam step over every parameter array of a Gaussian map in one launch,
// for the mapping loop that minimises the Eq. (12) loss (Sec. II-E; the paper
// leaves the optimiser unstated, the Gaussian-splatting lineage uses Adam).
// Per element, step t:  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
// p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
// Memory bound: 16 bytes read and 12 written per element; the five arrays
// are one flat index range, so one launch covers the map.
#include <cmath>

#include "api_range.hpp"
#include "common.hpp"

namespace mgs {
namespace {

struct AdamSeg {
    float *p, *m, *v;
    const float *g;
    float lr;
};

struct AdamArgs {
    AdamSeg seg[5];
    int64_t end[5];  // cumulative element counts of the active segments
    int nseg;
    float b1, b2, omb1, omb2, inv_bc1, inv_bc2, eps;
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
    const int64_t total = a.end[a.nseg - 1];
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < a.nseg && idx >= a.end[k]) ++k;
        const int64_t i = idx - (k ? a.end[k - 1] : 0);
        const AdamSeg &S = a.seg[k];
        const float g = S.g[i];
        const float m = a.b1 * S.m[i] + a.omb1 * g;
        const float v = a.b2 * S.v[i] + a.omb2 * (g * g);
        S.m[i] = m;
        S.v[i] = v;
        S.p[i] = S.p[i] - S.lr * (m * a.inv_bc1) / (sqrtf(v * a.inv_bc2) + a.eps);
    }
}

}  // namespace
}  // namespace mgs

using namespace mgs;

extern "C" mgs_status mgs_adam_step(const mgs_gaussians_out *params, int64_t n, int32_t sh_degree,
                                    const mgs_gaussian_grads *grads, const mgs_gaussians_out *exp_avg,
                                    const mgs_gaussians_out *exp_avg_sq, const mgs_adam_opts *opts, void *stream) {
    ApiRange api_range("mgs_adam_step");
    if (!params || !grads || !exp_avg || !exp_avg_sq || !opts) return MGS_ERR_INVALID_ARG;
    if (n < 0 || sh_degree < 0 || sh_degree > 3 || opts->step < 1) return MGS_ERR_INVALID_ARG;
    if (!(opts->beta1 >= 0.0f && opts->beta1 < 1.0f) || !(opts->beta2 >= 0.0f && opts->beta2 < 1.0f) ||
        !(opts->eps >= 0.0f) || !std::isfinite(opts->eps))
        return MGS_ERR_INVALID_ARG;
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(opts->lr[k])) return MGS_ERR_INVALID_ARG;
    if (n >= (int64_t(1) << 31)) return MGS_ERR_TOO_LARGE;
    const int64_t width[5] = {3, 3, 4, 1, 3 * (int64_t)(sh_degree + 1) * (sh_degree + 1)};
    float *const P[5] = {params->means, params->scales, params->quats, params->opac, params->sh};
    float *const M1[5] = {exp_avg->means, exp_avg->scales, exp_avg->quats, exp_avg->opac, exp_avg->sh};
    float *const M2[5] = {exp_avg_sq->means, exp_avg_sq->scales, exp_avg_sq->quats, exp_avg_sq->opac,
                          exp_avg_sq->sh};
    const float *const G[5] = {grads->d_means, grads->d_scales, grads->d_quats, grads->d_opac, grads->d_sh};
    AdamArgs a{};
    int64_t acc = 0;
    for (int k = 0; k < 5; ++k) {
        if (!G[k]) continue;  // no gradient: the group is left as it is
        if (n > 0 && (!P[k] || !M1[k] || !M2[k])) return MGS_ERR_INVALID_ARG;
        acc += n * width[k];
        a.seg[a.nseg] = AdamSeg{P[k], M1[k], M2[k], G[k], opts->lr[k]};
        a.end[a.nseg] = acc;
        ++a.nseg;
    }
    if (a.nseg == 0 || acc == 0) return MGS_OK;
    const double b1 = opts->beta1, b2 = opts->beta2;
    a.b1 = opts->beta1;
    a.b2 = opts->beta2;
    a.omb1 = (float)(1.0 - b1);
    a.omb2 = (float)(1.0 - b2);
    a.inv_bc1 = (float)(1.0 / (1.0 - std::pow(b1, opts->step)));
    a.inv_bc2 = (float)(1.0 / (1.0 - std::pow(b2, opts->step)));
    a.eps = opts->eps;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t blocks = std::min<int64_t>(ceil_div(acc, 256), 256 * 64);
    k_adam<<<(unsigned)blocks, 256, 0, s>>>(a);
    MGS_LAUNCHED();
    return MGS_OK;
}
