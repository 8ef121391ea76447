// Host sampler of the random cloud geometry omega (Sec. 3 and 3.1 of
// arXiv:1705.04374: centres uniform in the cloud, log-normal radii, optionally
// clipped).  Counter-based, so every (seed, term, index) is reproducible and
// independent of how samples are distributed over calls or devices.
// Built with -ffp-contract=off: the distance tests must not be fused.
#include <cmath>
#include <cstdint>

#include "ofm.h"
#include "ofm_error.h"

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
inline uint64_t mixer(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Rng {
    uint64_t state;
    uint64_t next() { state += kGolden; return mixer(state); }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

inline uint64_t first_output(uint64_t x) { return mixer(x + kGolden); }

}  // namespace

extern "C" int ofm_sample_cloud(const ofm_cloud_spec* spec, uint64_t seed, uint64_t term, uint64_t index,
                                double* out)
{
    if (!spec || !out) return ofm::fail(nullptr, OFM_EINVAL, "ofm_sample_cloud: null argument");
    const int d = spec->ndim;
    if (d < 1 || d > 3 || spec->n_bubbles < 0 || !(spec->cloud_radius > 0.0) || !(spec->r_median > 0.0))
        return ofm::fail(nullptr, OFM_EINVAL, "ofm_sample_cloud: bad cloud spec");
    const bool clip = spec->r_hi > 0.0;
    if (clip && !(spec->r_lo <= spec->r_median * 1e3 && spec->r_lo <= spec->r_hi))
        return ofm::fail(nullptr, OFM_EINVAL, "ofm_sample_cloud: bad radius range");
    Rng g{ first_output(first_output(first_output(seed) ^ term) ^ index) };
    const double twopi = 2.0 * M_PI;
    for (int b = 0; b < spec->n_bubbles; ++b) {
        int tries = 0;
        for (;;) {
            if (++tries > 100000)
                return ofm::fail(nullptr, OFM_EINFEASIBLE, "ofm_sample_cloud: no room for bubble %d", b);
            double v[3] = { 0.0, 0.0, 0.0 };
            for (;;) {
                for (int a = 0; a < d; ++a) v[a] = 2.0 * g.uniform() - 1.0;
                double n2 = v[0] * v[0];
                for (int a = 1; a < d; ++a) n2 = n2 + v[a] * v[a];
                if (n2 < 1.0) break;
            }
            double c[3] = { 0.0, 0.0, 0.0 };
            for (int a = 0; a < d; ++a) c[a] = spec->center[a] + spec->cloud_radius * v[a];
            double r;
            for (;;) {
                const double u1 = 1.0 - g.uniform();
                const double u2 = g.uniform();
                const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(twopi * u2);
                r = spec->r_median * std::exp(spec->r_sigma * z);
                if (!clip || (spec->r_lo <= r && r <= spec->r_hi)) break;
            }
            bool ok = true;
            for (int j = 0; j < b && ok; ++j) {
                const double* q = out + 4 * j;
                const double dx = c[0] - q[0];
                double d2 = dx * dx;
                for (int a = 1; a < d; ++a) {
                    const double da = c[a] - q[a];
                    d2 = d2 + da * da;
                }
                const double s = r + q[3];
                if (d2 < s * s) ok = false;
            }
            if (ok) {
                out[4 * b + 0] = c[0];
                out[4 * b + 1] = c[1];
                out[4 * b + 2] = c[2];
                out[4 * b + 3] = r;
                break;
            }
        }
    }
    return OFM_OK;
}
