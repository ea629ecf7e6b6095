// Plan-description checks (paper_2511_09165_amd/csrc/dmas_validate.hpp, the
// code dmas_plan_create runs before any device work) on the CPU, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py:
// every rejection path once, the defaults of a valid description, then a
// seeded fuzz over field values. Prints "ok <cases>" or the first mismatch
// and exits with status 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "../paper_2511_09165_amd/csrc/dmas_validate.hpp"

namespace {

constexpr int kChunk = 256;
int g_cases = 0;

struct Arrays {
    std::vector<double> mic, dirs;
    std::vector<float> taps, pulse;
    Arrays(int M, int D) : mic(3 * (size_t)M, 0.0), dirs(3 * (size_t)D, 0.0), taps(255, 0.01f), pulse(64, 1.0f)
    {
        for (int i = 0; i < M; ++i) mic[3 * i] = 0.01 * i;
        for (int p = 0; p < D; ++p) dirs[3 * p + 2] = 1.0;
    }
};

dmas_plan_desc_t base(Arrays &a, int M, int D)
{
    dmas_plan_desc_t d{};
    d.num_mics = M;
    d.num_samples = 1000;
    d.num_dirs = D;
    d.order = 2;
    d.use_cf = 1;
    d.geometry = DMAS_FARFIELD;
    d.mic_pos = a.mic.data();
    d.dirs = a.dirs.data();
    d.fs = 450e3;
    return d;
}

void expect(const dmas_plan_desc_t *d, dmas_status_t want, const char *what)
{
    char msg[512];
    dmas::DescValues v;
    const dmas_status_t got = dmas::validate_desc(d, kChunk, msg, sizeof msg, &v);
    ++g_cases;
    if (got != want) {
        std::printf("mismatch: %s: got %d want %d (%s)\n", what, (int)got, (int)want, got ? msg : "");
        std::exit(1);
    }
}

}  // namespace

int main()
{
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    Arrays a(8, 5);
    dmas_plan_desc_t d = base(a, 8, 5);

    {   // a valid description and its defaults
        char msg[64];
        dmas::DescValues v;
        if (dmas::validate_desc(&d, kChunk, msg, sizeof msg, &v) != DMAS_OK || v.c != 343.0 || v.cf_eps != 1e-20 ||
            v.fir_len != 63 || v.fir_fc != 5000.0 || v.env_decimation != 1) {
            std::printf("mismatch: defaults\n");
            return 1;
        }
        ++g_cases;
    }
    expect(nullptr, DMAS_ERR_INVALID_ARG, "NULL desc");
#define CASE(field, value, want)                  \
    do {                                          \
        dmas_plan_desc_t e = base(a, 8, 5);       \
        e.field = value;                          \
        expect(&e, want, #field " = " #value);    \
    } while (0)
    CASE(num_mics, 0, DMAS_ERR_INVALID_ARG);
    CASE(num_samples, 0, DMAS_ERR_INVALID_ARG);
    CASE(num_dirs, -3, DMAS_ERR_INVALID_ARG);
    CASE(order, 0, DMAS_ERR_INVALID_ARG);
    CASE(order, 9, DMAS_ERR_INVALID_ARG);
    CASE(num_samples, std::numeric_limits<int32_t>::max(), DMAS_ERR_INVALID_ARG);
    CASE(mic_pos, nullptr, DMAS_ERR_INVALID_ARG);
    CASE(dirs, nullptr, DMAS_ERR_INVALID_ARG);
    CASE(use_cf, 2, DMAS_ERR_INVALID_ARG);
    CASE(geometry, 7, DMAS_ERR_INVALID_ARG);
    CASE(in_dtype, 3, DMAS_ERR_INVALID_ARG);
    CASE(delay_mode, -1, DMAS_ERR_INVALID_ARG);
    CASE(ng_fp64, 2, DMAS_ERR_INVALID_ARG);
    CASE(compensated, 3, DMAS_ERR_INVALID_ARG);
    CASE(fs, 0.0, DMAS_ERR_INVALID_ARG);
    CASE(fs, nan, DMAS_ERR_INVALID_ARG);
    CASE(fs, inf, DMAS_ERR_INVALID_ARG);
    CASE(c, -343.0, DMAS_ERR_INVALID_ARG);
    CASE(c, inf, DMAS_ERR_INVALID_ARG);
    CASE(cf_eps, 1e-40, DMAS_ERR_INVALID_ARG);
    CASE(cf_eps, -1.0, DMAS_ERR_INVALID_ARG);
    CASE(fir_len, 64, DMAS_ERR_INVALID_ARG);
    CASE(fir_len, 257, DMAS_ERR_INVALID_ARG);
    CASE(fir_len, -1, DMAS_ERR_INVALID_ARG);
    CASE(fir_fc, 225e3, DMAS_ERR_INVALID_ARG);
    CASE(env_decimation, -2, DMAS_ERR_INVALID_ARG);
    CASE(env_decimation, 1001, DMAS_ERR_INVALID_ARG);
    CASE(env_decimation, 1000, DMAS_OK);
    CASE(mf_len, 5, DMAS_ERR_INVALID_ARG);
    CASE(order, 8, DMAS_OK);
    CASE(fir_len, 255, DMAS_OK);
    CASE(fir_len, 1, DMAS_OK);
#undef CASE
    {   // order above M; taps with a cut-off the default design would refuse
        dmas_plan_desc_t e = base(a, 8, 5);
        e.num_mics = 2;
        e.order = 3;
        expect(&e, DMAS_ERR_INVALID_ARG, "order > M");
        e = base(a, 8, 5);
        e.fir_taps = a.taps.data();
        e.fir_len = 255;
        e.fir_fc = 1e9;
        expect(&e, DMAS_OK, "explicit taps ignore fir_fc");
        a.taps[254] = (float)nan;
        expect(&e, DMAS_ERR_INVALID_ARG, "NaN tap");
        a.taps[254] = 0.01f;
        e = base(a, 8, 5);
        e.mf_pulse = a.pulse.data();
        e.mf_len = 64;
        expect(&e, DMAS_OK, "pulse");
        e.mf_len = 0;
        expect(&e, DMAS_ERR_INVALID_ARG, "pulse without length");
        e.mf_len = DMAS_MAX_MF_LEN + 1;
        expect(&e, DMAS_ERR_INVALID_ARG, "pulse too long");
        e.mf_len = 64;
        a.pulse[63] = (float)inf;
        expect(&e, DMAS_ERR_INVALID_ARG, "Inf in pulse");
        a.pulse[63] = 1.0f;
    }
    {   // geometry
        dmas_plan_desc_t e = base(a, 8, 5);
        a.mic[7] = nan;
        expect(&e, DMAS_ERR_INVALID_ARG, "NaN microphone");
        a.mic[7] = 0.0;
        a.dirs[14] = 2.0;
        expect(&e, DMAS_ERR_INVALID_ARG, "non-unit direction");
        e.geometry = DMAS_NEARFIELD;
        expect(&e, DMAS_OK, "voxel centre at 2 m");
        a.dirs[14] = 1.0e9;
        expect(&e, DMAS_ERR_INVALID_ARG, "delay span above 1e8 samples");
        a.dirs[14] = 1.0;
        e.geometry = DMAS_FARFIELD;
        a.mic[0] = 1.0e6;
        expect(&e, DMAS_ERR_INVALID_ARG, "far array");
        a.mic[0] = 0.0;
    }
    {   // combinations the library does not build
        dmas_plan_desc_t e = base(a, 8, 5);
        e.compensated = DMAS_ACCUM_KAHAN;
        expect(&e, DMAS_OK, "Kahan far field with CF");
        e.use_cf = 0;
        expect(&e, DMAS_ERR_UNSUPPORTED, "Kahan without CF");
        e = base(a, 8, 5);
        e.compensated = DMAS_ACCUM_F64;
        e.geometry = DMAS_NEARFIELD;
        expect(&e, DMAS_ERR_UNSUPPORTED, "FP64 sums in the near field");
        e = base(a, 8, 5);
        e.delay_mode = DMAS_DELAY_LINEAR;
        e.use_cf = 0;
        expect(&e, DMAS_ERR_UNSUPPORTED, "linear delays without CF");
        e.use_cf = 1;
        e.compensated = DMAS_ACCUM_KAHAN;
        expect(&e, DMAS_ERR_UNSUPPORTED, "linear delays with Kahan sums");
    }
    // fuzz: random field values (arrays always as large as the sizes say)
    std::mt19937 rng(2511091650u);
    std::uniform_int_distribution<int> small(-3, 12);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    for (int it = 0; it < 20000; ++it) {
        const int M = 1 + (int)(rng() % 40), D = 1 + (int)(rng() % 30);
        Arrays b(M, D);
        for (double &v : b.mic) v = (rng() % 50 == 0) ? nan : 0.1 * U(rng);
        for (int p = 0; p < D; ++p)
            for (int k = 0; k < 3; ++k) b.dirs[3 * p + k] = U(rng);
        dmas_plan_desc_t e = base(b, M, D);
        e.num_samples = (int)(rng() % 5000) - 10;
        e.order = small(rng);
        e.use_cf = small(rng) % 3;
        e.geometry = small(rng) % 3;
        e.in_dtype = small(rng) % 4;
        e.delay_mode = small(rng) % 3;
        e.compensated = small(rng) % 4;
        e.ng_fp64 = small(rng) % 3;
        e.fs = (rng() % 20 == 0) ? nan : 1e5 * (1.0 + U(rng));
        e.c = (rng() % 10 == 0) ? 0.0 : 343.0 * (1.0 + 0.5 * U(rng));
        e.fir_len = small(rng) * 21;
        e.fir_fc = 1e4 * (1.0 + U(rng));
        e.env_decimation = small(rng) * 100;
        if (rng() % 3 == 0) {
            e.fir_taps = b.taps.data();
            e.fir_len = 1 + 2 * (int)(rng() % 127);
        }
        if (rng() % 3 == 0) {
            e.mf_pulse = b.pulse.data();
            e.mf_len = (int)(rng() % 64);
        }
        char msg[512];
        dmas::DescValues v;
        const dmas_status_t st = dmas::validate_desc(&e, kChunk, msg, sizeof msg, &v);
        ++g_cases;
        if (st != DMAS_OK && st != DMAS_ERR_INVALID_ARG && st != DMAS_ERR_UNSUPPORTED) {
            std::printf("mismatch: fuzz case %d returned %d\n", it, (int)st);
            return 1;
        }
        if (st == DMAS_OK && (e.order < 1 || e.order > e.num_mics || v.fir_len % 2 == 0 || v.env_decimation < 1)) {
            std::printf("mismatch: fuzz case %d accepted an invalid description\n", it);
            return 1;
        }
    }
    std::printf("ok %d\n", g_cases);
    return 0;
}
