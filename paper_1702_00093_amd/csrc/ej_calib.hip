// Distortion diagnostics and parameter calibration.
//
// The paper studies how far the CGK embedding stretches edit distance
// (distortion = Hamming distance of the embeddings / edit distance, the best
// of r embeddings, Section 3.1) and how the truncation L moves the normalised
// Hamming distance Ham/L of similar and dissimilar pairs (Section 6), and
// picks r, z, m and L from those observations.  ej_embed_hamming measures the
// Hamming distances on the GPU; ej_calibrate turns them into a choice.
//
// Given a pair's embeddings under seed l at Hamming distance H over L
// symbols, a table of that seed (m coordinates drawn uniformly with
// replacement) gives the pair one key with probability q_l = (1 - H/L)^m,
// independently for each of the z tables of the seed (Section 3.2).  So the
// number of tables in which the pair collides is a sum of independent
// Bernoulli trials -- z with probability q_l for each seed l -- and
//   EmbedJoin:  P[candidate] = 1 - prod_l (1 - q_l)^z;
//   EmbedJoin+: P[some suffix pair counted >= T] >= P[the suffix pair of the
//               least Hamming distance counted >= T] (exact for one suffix),
// evaluated by dynamic programming over the tables (counts capped at T).
// Averaging over sampled pairs within K gives the expected recall; over
// pairs beyond K, the probability that a dissimilar pair becomes a
// candidate.  These expectations are over the LSH coordinate draws for the
// seeds' actual embeddings (the embeddings are the ones the join will use:
// R^l depends only on the seed and l).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ej_internal.h"

namespace ej {

namespace {

// Distribution of the number of agreeing tables, capped at T (dp[T] holds
// P[count >= T]), extended by one seed whose z tables agree each with
// probability q: a convolution with Binomial(z, q).
void add_seed(std::vector<double> &dp, std::vector<double> &nx, std::vector<double> &bin,
              uint32_t z, uint32_t T, double q) {
    bin.assign(z + 1, 0.0);
    for (uint32_t k = 0; k <= z; k++) {
        double c = 1.0;
        for (uint32_t i = 0; i < k; i++) c = c * (double)(z - i) / (double)(i + 1);
        bin[k] = c * pow(q, (double)k) * pow(1.0 - q, (double)(z - k));
    }
    nx.assign(T + 1, 0.0);
    for (uint32_t c = 0; c <= T; c++) {
        if (dp[c] == 0.0) continue;
        for (uint32_t k = 0; k <= z; k++) nx[std::min(T, c + k)] += dp[c] * bin[k];
    }
    dp.swap(nx);
}

uint32_t effective_L(const Prep &pp, uint32_t L_req) {
    uint64_t L = L_req;
    if (L == 0) L = pp.n ? (pp.total + pp.n - 1) / pp.n : 1;
    if (L > 3ull * pp.maxlen) L = 3ull * pp.maxlen;
    if (L == 0) L = 1;
    return (uint32_t)L;
}

}  // namespace

}  // namespace ej

using namespace ej;

extern "C" {

ej_status ej_embed_hamming(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                           uint32_t n, const ej_params *p, uint32_t delta,
                           const uint64_t *d_pairs, uint64_t count, uint32_t *d_ham) {
    if (!p || !d_offsets || (count && (!d_pairs || !d_ham))) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        if (p->r == 0 || p->r > 4096) fail(EJ_EINVAL, "r must be in 1..4096");
        if (n >= 0x80000000u) fail(EJ_EINVAL, "n must be below 2^31");
        const uint32_t kappa =
            delta ? std::max<uint32_t>(1u, (uint32_t)((p->K + (uint64_t)delta - 1) / delta)) : 1u;
        if ((uint64_t)kappa * kappa > 4096) fail(EJ_EUNSUPPORTED, "more than 64 suffixes per string");
        Prep pp;
        prepare(ctx, d_chars, d_offsets, n, p->L, pp, "h", nullptr, 0, 0, false);
        check_pairs(ctx, d_pairs, count, n, n);
        ej_params q = *p;
        q.z = 1;
        q.m = 1;
        Rand rd;
        draw_randomness(ctx, q, pp.L, pp.sigma, rd, "h");
        embed_hamming(ctx, pp, rd, d_pairs, count, kappa, delta, d_ham);
        sync(ctx);
    });
}

ej_status ej_calibrate(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                       const uint64_t *d_pairs, uint64_t count, const ej_calib_opts *o,
                       ej_calib_result *out, double *table) {
    if (!o || !out || !d_offsets || (count && !d_pairs)) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        memset(out, 0, sizeof(*out));
        if (o->r_max == 0 || o->r_max > 4096 || !o->nz || !o->nm || !o->nL || !o->z_list ||
            !o->m_list || !o->L_list)
            fail(EJ_EINVAL, "empty calibration grid");
        if (verify_lanes_for(o->K) == 0) fail(EJ_EUNSUPPORTED, "K above 2046 is not supported");
        for (uint32_t i = 0; i < o->nz; i++)
            if (o->z_list[i] == 0 || (uint64_t)o->z_list[i] * o->r_max > 4096)
                fail(EJ_EINVAL, "z must be positive and r_max*z at most 4096");
        for (uint32_t i = 0; i < o->nm; i++)
            if (o->m_list[i] == 0 || o->m_list[i] > 64) fail(EJ_EINVAL, "m must be in 1..64");
        if (n >= 0x80000000u) fail(EJ_EINVAL, "n must be below 2^31");
        if (o->reserved != 0) fail(EJ_EINVAL, "ej_calib_opts.reserved must be 0");
        const bool plus = o->delta != 0;
        const uint32_t kappa =
            plus ? std::max<uint32_t>(1u, (uint32_t)((o->K + (uint64_t)o->delta - 1) / o->delta))
                 : 1u;
        if ((uint64_t)kappa * kappa > 4096) fail(EJ_EUNSUPPORTED, "more than 64 suffixes per string");
        const uint32_t T = !plus ? 1u : (o->T ? o->T : (kappa > 1 ? 2u : 1u));
        Prep pp;
        prepare(ctx, d_chars, d_offsets, n, 0, pp, "h", nullptr, 0, 0, false);
        check_pairs(ctx, d_pairs, count, n, n);
        // exact distances of the sample pairs: within K or not
        std::vector<int32_t> dist(count);
        if (count) {
            RowMasks masks;
            build_masks(ctx, pp.d_codes, d_offsets, pp.base, n, pp.total, pp.sigma, masks, "h");
            int32_t *d_dist = ws<int32_t>(ctx, "h_dist", count);
            verify(ctx, pp.d_codes, d_offsets, pp.base, pp.sigma, pp.maxlen, masks, d_pairs, count,
                   o->K, nullptr, d_dist);
            EJ_HIP(hipMemcpyAsync(dist.data(), d_dist, 4 * count, hipMemcpyDeviceToHost,
                                  ctx->stream));
            sync(ctx);
        }
        // sample pairs the short pass (exact_len) makes candidates with certainty
        std::vector<char> certain(count, 0);
        if (o->exact_len && count) {
            std::vector<uint32_t> len(n);
            std::vector<uint64_t> pr(count);
            EJ_HIP(hipMemcpyAsync(len.data(), pp.d_len, 4ull * n, hipMemcpyDeviceToHost,
                                  ctx->stream));
            EJ_HIP(hipMemcpyAsync(pr.data(), d_pairs, 8 * count, hipMemcpyDeviceToHost,
                                  ctx->stream));
            sync(ctx);
            for (uint64_t e = 0; e < count; e++)
                certain[e] = len[pr[e] >> 32] <= o->exact_len &&
                             len[(uint32_t)pr[e]] <= o->exact_len;
        }
        std::vector<char> similar(count);
        for (uint64_t e = 0; e < count; e++) {
            similar[e] = dist[e] >= 0 && (uint32_t)dist[e] <= o->K;
            if (similar[e])
                out->n_similar++;
            else
                out->n_dissimilar++;
        }
        const double avg_len = n ? (double)pp.total / n : 0.0;
        const uint32_t R = o->r_max;
        uint32_t *d_ham = ws<uint32_t>(ctx, "h_ham", count * R);
        std::vector<uint32_t> ham(count * R);
        std::vector<double> q(R), dp, nx, bin;
        std::vector<double> rec(R), fal(R);
        double best_work = 0.0;
        out->best_recall = 0.0;
        for (uint32_t li = 0; li < o->nL; li++) {
            const uint32_t L = effective_L(pp, o->L_list[li]);
            ej_params pr;
            memset(&pr, 0, sizeof(pr));
            pr.r = R;
            pr.z = 1;
            pr.m = 1;
            pr.seed = o->seed;
            Rand rd;
            draw_randomness(ctx, pr, L, pp.sigma, rd, "h");
            if (count) {
                embed_hamming(ctx, pp, rd, d_pairs, count, kappa, o->delta, d_ham);
                EJ_HIP(hipMemcpyAsync(ham.data(), d_ham, 4 * count * R, hipMemcpyDeviceToHost,
                                      ctx->stream));
                sync(ctx);
            }
            for (uint32_t zi = 0; zi < o->nz; zi++) {
                const uint32_t z = o->z_list[zi];
                for (uint32_t mi = 0; mi < o->nm; mi++) {
                    const uint32_t m = o->m_list[mi];
                    std::fill(rec.begin(), rec.end(), 0.0);
                    std::fill(fal.begin(), fal.end(), 0.0);
                    for (uint64_t e = 0; e < count; e++) {
                        for (uint32_t l = 0; l < R; l++)
                            q[l] = pow(1.0 - (double)ham[e * R + l] / L, (double)m);
                        // every r in 1..R: the first r seeds, one seed added at a time
                        double miss = 1.0;
                        if (T > 1) {
                            dp.assign(T + 1, 0.0);
                            dp[0] = 1.0;
                        }
                        for (uint32_t r = 1; r <= R; r++) {
                            double pc;
                            if (T == 1) {
                                miss *= pow(1.0 - q[r - 1], (double)z);
                                pc = 1.0 - miss;
                            } else {
                                add_seed(dp, nx, bin, z, T, q[r - 1]);
                                pc = dp[T];
                            }
                            (similar[e] ? rec : fal)[r - 1] += certain[e] ? 1.0 : pc;
                        }
                    }
                    for (uint32_t r = 1; r <= R; r++) {
                        const double recall = out->n_similar ? rec[r - 1] / out->n_similar : 0.0;
                        const double frate = out->n_dissimilar ? fal[r - 1] / out->n_dissimilar : 0.0;
                        // predicted work per string, in 32-bit operations: the walk (3 per
                        // step, at most L steps per suffix and seed), the key hash (about 10
                        // per sampled symbol), bucketing and pair walk (about 60 per table
                        // entry), and the verification of false candidates (10 per 32-cell
                        // band word, K+1 cells wide, rejected after about 2K + 64 columns)
                        const double walks = (double)r * kappa;
                        const double work = 3.0 * walks * L + 10.0 * walks * z * m +
                                            60.0 * walks * z +
                                            frate * (n ? n - 1 : 0) / 2.0 * 10.0 *
                                                ((o->K + 1) / 32.0) *
                                                std::min(2.0 * o->K + 64.0, avg_len);
                        if (table) {
                            double *t = table + ((((uint64_t)li * R + (r - 1)) * o->nz + zi) *
                                                     o->nm + mi) * 3;
                            t[0] = recall;
                            t[1] = frate;
                            t[2] = work;
                        }
                        out->best_recall = std::max(out->best_recall, recall);
                        if (recall >= o->target_recall && (out->r == 0 || work < best_work)) {
                            best_work = work;
                            out->r = r;
                            out->z = z;
                            out->m = m;
                            out->L = L;
                            out->recall = recall;
                            out->false_rate = frate;
                            out->work = work;
                        }
                    }
                }
            }
        }
    });
}

}  // extern "C"
