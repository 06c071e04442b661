/*
 * pa_oracle.h -- plain, single-threaded FP64 CPU oracle for the K-means-seeded
 * elitist 2D genetic algorithm for pilot assignment (Alqudah & Khokhar,
 * "Efficient Parallel Implementation of the Pilot Assignment Problem in
 * Massive MIMO Systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this library; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with the
 * GPU library.
 *
 * Conventions (all arrays dense, row-major, caller-owned):
 *   beta[(l*L + j)*K + k]  large-scale fading of user k of cell j seen at the
 *                          base station of cell l (Sec. 3.1, Eq. 1-2).
 *   pop[(n*L + j)*K + k]   pilot index (0..K-1) used by user k of cell j in
 *                          chromosome n; every row j is a permutation (Sec. 4.1).
 *   user_xy[((j*K)+k)*2+d] user position (metres), bs_xy[j*2+d] BS position.
 *
 * Functions return 0 on success and a negative value on invalid input.
 */
#ifndef PA_ORACLE_H
#define PA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PAO_SE_ASYMPTOTIC = 0, PAO_SE_FINITE_M = 1 };

enum {
  PAO_TAG_SELECT = 0x01,
  PAO_TAG_MUT_DECIDE = 0x02,
  PAO_TAG_MUT_PARTNER = 0x03,
  PAO_TAG_INIT_DECIDE = 0x10,
  PAO_TAG_INIT_PARTNER = 0x11,
  PAO_TAG_INIT_SHUFFLE = 0x12
};

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void pao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Word `idx` of the stream (seed; c0, c1, c2, tag). */
uint32_t pao_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                  uint32_t idx);
uint32_t pao_bounded(uint32_t w, uint32_t n);
uint64_t pao_threshold(double p);

/* Sum spectral efficiency (Eq. 5-7) of n chromosomes, FP64. */
int pao_fitness(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                const double *beta, const uint8_t *pop, int32_t n, double *fit);
/* objective 0 = pao_fitness; 1 = the smallest per-user SINR (max-min SIR);
 * 2 = minus the inter-cluster interference of Eq. 8. */
int pao_fitness_obj(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                    int32_t objective, const double *beta, const uint8_t *pop, int32_t n,
                    double *fit);
/* Per-(cell, user) SE terms of one chromosome, [L][K], before the pre-log. */
int pao_se_terms(int32_t L, int32_t K, int32_t se_mode, double M, double rho,
                 const double *beta, const uint8_t *chrom, double *se);
/* Per-(cell, user) SINR of one chromosome, [L][K]. */
int pao_sinr_terms(int32_t L, int32_t K, int32_t se_mode, double M, double rho,
                   const double *beta, const uint8_t *chrom, double *sinr);

/* Ranking: order[0..n) = indices best first; returns 0. */
int pao_rank(const double *fit, int32_t n, int32_t *order);

/* K-means seed chromosome (integer Lloyd on in-cell offsets, k = K). */
int pao_kmeans_seed(int32_t L, int32_t K, const double *user_xy, const double *bs_xy,
                    uint8_t *seed_chrom, int32_t *centroids /*[K][2] or NULL*/,
                    int32_t *labels /*[L*K] or NULL*/, int32_t *iters /*or NULL*/);
/* Initial population [N][L][K]; seed_chrom may be NULL when kmeans_frac == 0. */
int pao_init_pop(int32_t L, int32_t K, int32_t N, double kmeans_frac, double p_init,
                 uint64_t seed, uint32_t instance_id, const uint8_t *seed_chrom, uint8_t *pop);
/* Mutation codes [L*K] of the child in `slot` at generation `gen`: k'+1 for a
 * gene (j, k) that swaps with user k' of its cell, 0 otherwise (decision
 * words bit-sliced over groups of 32 genes, partners by hit rank). */
int pao_mutation_codes(int32_t L, int32_t K, double p_mut, uint64_t seed, uint32_t slot,
                       uint32_t gen, uint32_t instance_id, uint8_t *codes);
/* One generation: elitism, tournament selection, row crossover, swap mutation. */
int pao_ga_step(int32_t L, int32_t K, int32_t N, int32_t E, double p_cross, double p_mut,
                uint64_t seed, uint32_t instance_id, uint32_t gen, const uint8_t *pop_in,
                const double *fit_in, uint8_t *pop_out);
/* Whole solve; best[L*K], trace[gens+1] (may be NULL), final_pop[N*L*K] (may be NULL). */
int pao_solve(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
              const double *beta, const double *user_xy, const double *bs_xy, int32_t N,
              int32_t gens, int32_t E, double p_cross, double p_mut, double kmeans_frac,
              double p_init, uint64_t seed, uint32_t instance_id, uint8_t *best,
              double *best_fit, double *trace, uint8_t *final_pop);
/* Island GA (PK-means GA, Alg. 2): K-means of the population into C islands
 * (chromosomes as points of Z^{LK}, farthest-point start from the best, at
 * most max_iters Lloyd iterations), labels[N] and centroids[C][L*K]. */
int pao_pop_kmeans(int32_t L, int32_t K, int32_t N, int32_t C, const uint8_t *pop,
                   const double *fit, int32_t max_iters, int32_t *labels, uint8_t *centroids,
                   int32_t *iters);
/* One generation of every island (members = positions labelled c). */
int pao_island_step(int32_t L, int32_t K, int32_t N, int32_t E, int32_t C,
                    const int32_t *labels, double p_cross, double p_mut, uint64_t seed,
                    uint32_t instance_id, uint32_t gen, const uint8_t *pop_in,
                    const double *fit_in, uint8_t *pop_out);
/* Whole island solve: K-means of the population at generation 0 and every
 * recluster_every generations (0 = only at 0). */
int pao_island_solve(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                     const double *beta, const double *user_xy, const double *bs_xy, int32_t N,
                     int32_t gens, int32_t E, double p_cross, double p_mut, double kmeans_frac,
                     double p_init, uint64_t seed, uint32_t instance_id, int32_t C,
                     int32_t recluster_every, int32_t max_iters, uint8_t *best, double *best_fit,
                     double *trace, uint8_t *final_pop, int32_t *final_labels);
/* Exhaustive search over the K!^(L-1) classes (row 0 fixed to the identity). */
int pao_bruteforce(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                   const double *beta, uint8_t *best, double *best_fit, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif
