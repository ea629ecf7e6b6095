// Checks of a plan description that dmas_plan_create makes before any device
// work, free of device calls so that a CPU build with sanitizers runs the same
// code in tests. Host arrays are read within the sizes the description states
// (3 M microphone and 3 D direction coordinates, fir_len taps, mf_len pulse
// samples), as the C ABI's contract says.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "../../include/dmas.h"

namespace dmas {

// Effective values of the fields whose 0 selects a default.
struct DescValues {
    double c = 343.0;
    double cf_eps = 1e-20;
    double fir_fc = 5000.0;
    int fir_len = 63;
    int env_decimation = 1;
};

namespace detail {

inline dmas_status_t desc_fail(char *msg, size_t len, dmas_status_t st, const char *fmt, ...)
{
    if (msg && len) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(msg, len, fmt, ap);
        va_end(ap);
    }
    return st;
}

inline bool finite_all(const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace detail

// DMAS_OK, or the status of the first problem found with its message in msg
// (len bytes). `chunk` is the kernels' samples per chunk (the record length
// must leave room for the envelope's halo and chunk rounding in 32-bit
// sample indices). On success *out holds the effective defaults.
inline dmas_status_t validate_desc(const dmas_plan_desc_t *d, int chunk, char *msg, size_t len, DescValues *out)
{
    using detail::desc_fail;
    if (!d) return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "desc is NULL");
    const int M = d->num_mics, T = d->num_samples, D = d->num_dirs, n = d->order;
    if (M < 1 || T < 1 || D < 1)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "sizes must be >= 1 (M=%d T=%d D=%d)", M, T, D);
    if (n < 1 || n > DMAS_MAX_ORDER)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "order %d outside 1..%d", n, DMAS_MAX_ORDER);
    if (n > M)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "order %d exceeds the number of microphones %d", n, M);
    if ((int64_t)T + 2 * DMAS_MAX_FIR_LEN + 4 * (int64_t)chunk > INT32_MAX / 2)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "num_samples %d too large", T);
    if (!d->mic_pos || !d->dirs) return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "mic_pos or dirs is NULL");
    if (d->use_cf != 0 && d->use_cf != 1) return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "use_cf must be 0 or 1");
    if (d->geometry != DMAS_FARFIELD && d->geometry != DMAS_NEARFIELD)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "unknown geometry %d", d->geometry);
    if (d->in_dtype != DMAS_F32 && d->in_dtype != DMAS_F16 && d->in_dtype != DMAS_BF16)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "unknown in_dtype %d", d->in_dtype);
    if (d->delay_mode != DMAS_DELAY_NEAREST && d->delay_mode != DMAS_DELAY_LINEAR)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "unknown delay_mode %d", d->delay_mode);
    if (d->ng_fp64 != 0 && d->ng_fp64 != 1) return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "ng_fp64 must be 0 or 1");
    if (d->compensated < DMAS_ACCUM_F32 || d->compensated > DMAS_ACCUM_F64)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "compensated must be 0 (FP32), 1 (Kahan) or 2 (FP64)");
    if (!(d->fs > 0.0) || !std::isfinite(d->fs)) return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "fs must be > 0");
    DescValues v;
    v.c = d->c == 0.0 ? 343.0 : d->c;
    if (!(v.c > 0.0) || !std::isfinite(v.c)) return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "c must be > 0");
    v.cf_eps = d->cf_eps == 0.0 ? 1e-20 : d->cf_eps;
    if (!(v.cf_eps > 0.0) || !std::isfinite(v.cf_eps) || v.cf_eps < 1.1754944e-38)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "cf_eps must be a positive normal FP32 value");
    v.fir_len = d->fir_len == 0 ? 63 : d->fir_len;
    if (v.fir_len < 1 || v.fir_len > DMAS_MAX_FIR_LEN || (v.fir_len % 2) == 0)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "fir_len %d must be odd in 1..%d", v.fir_len,
                         DMAS_MAX_FIR_LEN);
    v.fir_fc = d->fir_fc == 0.0 ? 5000.0 : d->fir_fc;
    if (!d->fir_taps && !(v.fir_fc > 0.0 && v.fir_fc < 0.5 * d->fs))
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "fir_fc must lie in (0, fs/2)");
    if (!detail::finite_all(d->mic_pos, 3 * (size_t)M) || !detail::finite_all(d->dirs, 3 * (size_t)D))
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "geometry contains NaN or Inf");
    if (d->geometry == DMAS_FARFIELD) {
        for (int p = 0; p < D; ++p) {
            const double *u = d->dirs + 3 * (size_t)p;
            const double nrm = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (std::fabs(nrm - 1.0) > 1e-6)
                return desc_fail(msg, len, DMAS_ERR_INVALID_ARG,
                                 "far-field direction %d is not a unit vector (|u| = %.9g)", p, nrm);
        }
    }
    {
        // Steering delays are whole samples in 32-bit integers: keep |fs*tau| far from overflow.
        double rmax = 0, vmax = 0;
        for (int i = 0; i < M; ++i) {
            const double *r = d->mic_pos + 3 * (size_t)i;
            rmax = std::max(rmax, std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]));
        }
        if (d->geometry == DMAS_NEARFIELD)
            for (int q = 0; q < D; ++q) {
                const double *p = d->dirs + 3 * (size_t)q;
                vmax = std::max(vmax, std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
            }
        const double span = d->fs * (d->geometry == DMAS_NEARFIELD ? 2.0 * (rmax + vmax) : rmax) / v.c;
        if (!(span < 1.0e8))
            return desc_fail(msg, len, DMAS_ERR_INVALID_ARG,
                             "geometry spans %.3g samples of delay; at most 1e8 is supported", span);
    }
    if (d->compensated && (d->geometry != DMAS_FARFIELD || !d->use_cf))
        return desc_fail(msg, len, DMAS_ERR_UNSUPPORTED,
                         "Kahan and FP64 accumulation are built for far field with CF only");
    if (d->delay_mode == DMAS_DELAY_LINEAR && !d->use_cf)
        return desc_fail(msg, len, DMAS_ERR_UNSUPPORTED, "linear delays are built with CF only");
    if (d->delay_mode == DMAS_DELAY_LINEAR && d->compensated)
        return desc_fail(msg, len, DMAS_ERR_UNSUPPORTED, "linear delays are built with FP32 accumulation only");
    v.env_decimation = d->env_decimation == 0 ? 1 : d->env_decimation;
    if (v.env_decimation < 1 || v.env_decimation > T)
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "env_decimation %d must lie in 1..T", v.env_decimation);
    if (d->mf_len < 0 || d->mf_len > DMAS_MAX_MF_LEN || (d->mf_pulse && d->mf_len < 1) ||
        (!d->mf_pulse && d->mf_len))
        return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "mf_len must be 1..%d with mf_pulse, 0 without",
                         DMAS_MAX_MF_LEN);
    if (d->mf_pulse) {
        for (int k = 0; k < d->mf_len; ++k)
            if (!std::isfinite(d->mf_pulse[k]))
                return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "mf_pulse contains NaN or Inf");
    }
    if (d->fir_taps) {
        for (int k = 0; k < v.fir_len; ++k)
            if (!std::isfinite(d->fir_taps[k]))
                return desc_fail(msg, len, DMAS_ERR_INVALID_ARG, "fir_taps contain NaN or Inf");
    }
    if (out) *out = v;
    return DMAS_OK;
}

}  // namespace dmas
