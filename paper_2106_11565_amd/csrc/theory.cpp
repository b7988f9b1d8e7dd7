// Parameters from the method's theory (Section 5 and its proofs): host
// arithmetic only.
//
// Group testing (Lemma 1 and the cellwise rate bounds): with B = 2 sqrt(N)
// groups per repetition, tests of true positive rate p and false positive
// rate q answer the randomized nearest-neighbour problem with failure
// probability delta when q = N^-1/2, p = 1 - delta / (2R) and
//   R = ln(1/delta) / (ln(4.80 sqrt N) - ln(2 e^2 + 3.44 sqrt N)),
// for N >= 150 and delta small enough that R >= 10 ln N.
//
// Each test is a distance-sensitive Bloom filter over the N/B points of a
// group (Theorem 1, with the threshold as a fraction t/m of the m arrays):
// concatenating K hashes (the paper's L), positives collide in an array with
// probability at least s_K^K and negatives at most (N/B) s_{K+1}^K.  K is the
// smallest integer with s_K^K >= 2 (N/B) s_{K+1}^K, the threshold ratio t/m
// the midpoint of the two, and the filter then errs with probability at most
//   alpha = exp(-2 m ((s_K^K - (N/B) s_{K+1}^K) / 2)^2)
// on either side.  The number of arrays m (tables, the paper's m) is the
// smallest with alpha <= min(q, 1 - p).  The paper's closed form
// m = -8 ln(min(q, 1 - p)) N^gamma, with the query's stability
// gamma = ln s_K / (ln s_{K+1} - ln s_K), takes K real-valued; it is
// reported beside the m that the integer K needs.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "flinng_internal.h"

namespace flinng {

static void theory(uint64_t N, double sk, double sk1, double delta, flinng_theory &o) {
    if (N < 2) fail(FLINNG_EINVAL, "N must be at least 2");
    if (!(sk > 0.0 && sk < 1.0 && sk1 > 0.0 && sk1 < sk))
        fail(FLINNG_EINVAL, "similarities must satisfy 0 < s_k1 < s_k < 1");
    if (!(delta > 0.0 && delta < 1.0)) fail(FLINNG_EINVAL, "delta must lie in (0, 1)");
    const double n = (double)N, rn = std::sqrt(n);
    const double den = std::log(4.80 * rn) - std::log(2.0 * std::exp(2.0) + 3.44 * rn);
    if (!(den > 0.0)) fail(FLINNG_EINVAL, "N too small for the repetition bound (needs N > 118)");
    std::memset(&o, 0, sizeof(o));
    // groups and repetitions
    const double Bd = std::max(1.0, std::floor(2.0 * rn + 0.5));
    o.B = (uint32_t)std::min<double>(Bd, (double)N);
    o.R_real = std::log(1.0 / delta) / den;
    if (o.R_real > 1e9) fail(FLINNG_EINVAL, "R out of range");
    o.R = (uint32_t)std::ceil(o.R_real);
    if (o.R < 1) o.R = 1;
    o.q = 1.0 / rn;
    o.one_minus_p = delta / (2.0 * (double)o.R);  // kept apart: p rounds to 1 for tiny delta
    o.p = 1.0 - o.one_minus_p;
    o.conditions_met = (N >= 150 && o.R_real >= 10.0 * std::log(n)) ? 1u : 0u;
    // hashes per table: smallest K >= 1 with s_K^K >= 2 (N/B) s_{K+1}^K,
    // i.e. K (ln s_K - ln s_{K+1}) >= ln(2 N / B)
    const double per = n / (double)o.B;
    const double gap = std::log(sk) - std::log(sk1);
    double Kd = std::ceil(std::log(2.0 * per) / gap);
    if (Kd < 1.0) Kd = 1.0;
    if (Kd > 4e9) fail(FLINNG_EINVAL, "similarities too close: K out of range");
    uint32_t K = (uint32_t)Kd;
    // the rounding of the logarithms: settle on the smallest K that holds
    auto holds = [&](uint32_t k) {
        return k * std::log(sk) >= std::log(2.0 * per) + k * std::log(sk1);
    };
    while (K > 1 && holds(K - 1)) --K;
    while (!holds(K)) ++K;
    o.K = K;
    o.t_over_m_low = per * std::pow(sk1, (double)K);
    o.t_over_m_high = std::pow(sk, (double)K);
    const double diff = o.t_over_m_high - o.t_over_m_low;
    const double target = std::min(o.q, o.one_minus_p);
    o.gamma = std::log(sk) / (std::log(sk1) - std::log(sk));
    o.m_paper = -8.0 * std::log(target) * std::pow(n, o.gamma);
    // smallest m with exp(-2 m (diff / 2)^2) <= target
    const double m_need = -2.0 * std::log(target) / (diff * diff);
    if (!(m_need < 4e9)) fail(FLINNG_EINVAL, "tables out of range");
    uint32_t m = (uint32_t)std::ceil(m_need);
    if (m < 1) m = 1;
    auto alpha_of = [&](uint32_t mm) { return std::exp(-2.0 * (double)mm * (diff / 2.0) * (diff / 2.0)); };
    while (m > 1 && alpha_of(m - 1) <= target) --m;
    while (alpha_of(m) > target) ++m;
    o.L = m;
    o.alpha = alpha_of(m);
    o.t_real = (double)m * (o.t_over_m_low + o.t_over_m_high) / 2.0;
    o.t = (uint32_t)std::ceil(o.t_real);
}

}  // namespace flinng

using namespace flinng;

extern "C" int flinng_theory_params(uint64_t N, double s_k, double s_k1, double delta,
                                    flinng_theory *out) {
    try {
        if (!out) fail(FLINNG_EINVAL, "NULL argument");
        theory(N, s_k, s_k1, delta, *out);
        set_last_error("");
        return FLINNG_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (...) {
        set_last_error("internal error");
        return FLINNG_EDEVICE;
    }
}
