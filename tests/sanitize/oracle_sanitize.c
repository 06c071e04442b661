/* Drives every oracle function on small inputs, the edge cases of each
 * (one cell, one user, E = 0 and E = N, one island, islands as many as
 * chromosomes) and inputs it must reject (rows that are not permutations,
 * unknown objectives), so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks every array access and integer operation
 * of the oracle.  Exit status 0 and "ok" when every call returned what it
 * must; the sanitizers abort on the first error they find. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/pa_oracle.h"

static uint64_t lcg_state = 0x9E3779B97F4A7C15ull;
static double unit(void) {
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) abort();
  return p;
}

/* a random population of permutation rows */
static void rand_pop(int L, int K, int N, uint8_t *pop) {
  for (int c = 0; c < N; ++c)
    for (int j = 0; j < L; ++j) {
      uint8_t *row = pop + ((size_t)c * L + j) * K;
      for (int k = 0; k < K; ++k) row[k] = (uint8_t)k;
      for (int k = K - 1; k > 0; --k) {
        int r = (int)(unit() * (k + 1));
        if (r > k) r = k;
        uint8_t t = row[k];
        row[k] = row[r];
        row[r] = t;
      }
    }
}

static void one_shape(int L, int K, int N, int E, int G, int C) {
  const size_t LK = (size_t)L * K;
  double *beta = xmalloc(sizeof(double) * L * LK);
  double *uxy = xmalloc(sizeof(double) * LK * 2), *bxy = xmalloc(sizeof(double) * L * 2);
  for (size_t i = 0; i < (size_t)L * LK; ++i) beta[i] = exp(-8.0 * unit()) + 1e-6;
  for (int j = 0; j < L; ++j) {
    bxy[2 * j] = 1000.0 * j;
    bxy[2 * j + 1] = -500.0 * j;
    for (int k = 0; k < K; ++k) {
      uxy[(j * K + k) * 2] = bxy[2 * j] + 400.0 * (unit() - 0.5);
      uxy[(j * K + k) * 2 + 1] = bxy[2 * j + 1] + 400.0 * (unit() - 0.5);
    }
  }
  uint8_t *pop = xmalloc(LK * N), *next = xmalloc(LK * N), *best = xmalloc(LK);
  uint8_t *seed = xmalloc(LK), *codes = xmalloc(LK), *cent = xmalloc(LK * C);
  double *fit = xmalloc(sizeof(double) * N), *terms = xmalloc(sizeof(double) * LK);
  double *trace = xmalloc(sizeof(double) * (G + 1));
  int32_t *order = xmalloc(sizeof(int32_t) * N), *labels = xmalloc(sizeof(int32_t) * N);
  int32_t *kcent = xmalloc(sizeof(int32_t) * K * 2), *klab = xmalloc(sizeof(int32_t) * LK);
  int32_t iters = 0;
  double bf = 0.0;
  rand_pop(L, K, N, pop);
  /* one cell: finite-M only (the asymptotic SIR of a lone cell is unbounded) */
  for (int m = L >= 2 ? 0 : 1; m < 2; ++m) {
    EXPECT(pao_fitness(L, K, 196, m, 64.0, 10.0, beta, pop, N, fit) == 0);
    for (int obj = 0; obj < 3; ++obj)
      EXPECT(pao_fitness_obj(L, K, 0, m, 64.0, 10.0, obj, beta, pop, N, fit) == 0);
    EXPECT(pao_se_terms(L, K, m, 64.0, 10.0, beta, pop, terms) == 0);
    EXPECT(pao_sinr_terms(L, K, m, 64.0, 10.0, beta, pop, terms) == 0);
  }
  EXPECT(pao_fitness_obj(L, K, 0, 1, 64.0, 10.0, 3, beta, pop, N, fit) != 0);
  /* a row that is not a permutation is rejected */
  if (K >= 2) {
    memcpy(next, pop, LK);
    next[0] = next[1];
    EXPECT(pao_fitness(L, K, 0, 1, 64.0, 10.0, beta, next, 1, fit) != 0);
  }
  for (int c = 0; c < N; ++c) fit[c] = unit() < 0.1 ? NAN : (unit() < 0.2 ? 0.5 : unit());
  EXPECT(pao_rank(fit, N, order) == 0);
  EXPECT(pao_kmeans_seed(L, K, uxy, bxy, seed, kcent, klab, &iters) == 0);
  EXPECT(pao_init_pop(L, K, N, 0.5, 0.1, 7, 3, seed, next) == 0);
  EXPECT(pao_init_pop(L, K, N, 0.0, 0.1, 7, 3, NULL, next) == 0);
  for (int s = 0; s < N; s += 1 + N / 4) {
    EXPECT(pao_mutation_codes(L, K, 0.05, 7, (uint32_t)s, 2, 3, codes) == 0);
    EXPECT(pao_mutation_codes(L, K, 1.0, 7, (uint32_t)s, 2, 3, codes) == 0);
  }
  for (int e = 0; e <= 2; ++e) {
    const int EE = e == 0 ? 0 : (e == 1 ? E : N);
    EXPECT(pao_ga_step(L, K, N, EE, 0.8, 0.05, 7, 3, 1, pop, fit, next) == 0);
    EXPECT(pao_ga_step(L, K, N, EE, 1.0, 1.0, 7, 3, 1, pop, fit, next) == 0);
  }
  if (L >= 2) {
    EXPECT(pao_solve(L, K, 196, 0, 1.0, 1.0, beta, uxy, bxy, N, G, E, 0.8, 0.05, 0.5, 0.1, 7, 3,
                     best, &bf, trace, next) == 0);
    EXPECT(pao_solve(L, K, 0, 1, 64.0, 10.0, beta, NULL, NULL, N, G, E, 0.8, 0.05, 0.0, 0.1, 7,
                     3, best, &bf, NULL, NULL) == 0);
  }
  for (int c = 1; c <= C; c = c == C ? C + 1 : (c * 2 > C ? C : c * 2)) {
    EXPECT(pao_pop_kmeans(L, K, N, c, pop, fit, 20, labels, cent, &iters) == 0);
    EXPECT(pao_pop_kmeans(L, K, N, c, pop, fit, 1, labels, cent, NULL) == 0);
    EXPECT(pao_island_step(L, K, N, E, c, labels, 0.8, 0.05, 7, 3, 1, pop, fit, next) == 0);
    EXPECT(pao_island_step(L, K, N, 0, c, labels, 0.8, 0.05, 7, 3, 1, pop, fit, next) == 0);
    if (L >= 2)
      EXPECT(pao_island_solve(L, K, 196, 0, 1.0, 1.0, beta, uxy, bxy, N, G, E, 0.8, 0.05, 0.5,
                              0.1, 7, 3, c, 3, 20, best, &bf, trace, next, labels) == 0);
  }
  if (L >= 2 && L <= 3 && K <= 3) {
    int64_t count = 0;
    EXPECT(pao_bruteforce(L, K, 0, 0, 1.0, 1.0, beta, best, &bf, &count) == 0);
  }
  free(beta); free(uxy); free(bxy); free(pop); free(next); free(best); free(seed); free(codes);
  free(cent); free(fit); free(terms); free(trace); free(order); free(labels); free(kcent);
  free(klab);
}

int main(void) {
  uint32_t ctr[4] = {0, 1, 2, 3}, key[2] = {4, 5}, out[4];
  pao_philox4x32_10(ctr, key, out);
  (void)pao_word(0xFFFFFFFFFFFFFFFFull, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFF, 0xFFFFFFFFu);
  EXPECT(pao_bounded(0xFFFFFFFFu, 0xFFFFFFFFu) < 0xFFFFFFFFu);
  EXPECT(pao_threshold(1.0) == ((uint64_t)1 << 32) && pao_threshold(-1.0) == 0);
  EXPECT(pao_threshold(NAN) == 0);
  /* (L, K, N, E, G, C) */
  const int shapes[][6] = {{1, 1, 4, 1, 3, 1},  {1, 5, 9, 2, 3, 3},    {2, 1, 6, 2, 4, 2},
                           {2, 2, 7, 3, 5, 7},  {3, 3, 20, 2, 6, 5},   {5, 8, 33, 4, 4, 4},
                           {7, 4, 50, 2, 5, 5}, {4, 33, 17, 1, 2, 16}, {3, 64, 5, 5, 2, 2}};
  for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
    one_shape(shapes[s][0], shapes[s][1], shapes[s][2], shapes[s][3], shapes[s][4], shapes[s][5]);
  if (failures) {
    fprintf(stderr, "%d unexpected return values\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
