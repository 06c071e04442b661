/*
 * pa_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Written from the paper: system model Sec. 3.1 (Eq. 1-2), uplink spectral
 * efficiency Sec. 3.2 (Eq. 3-6), problem formulation Sec. 3.3 (Eq. 7),
 * chromosome encoding and K-means seeding Sec. 4.1, Alg. 1, elitism
 * (contribution 1 in Sec. 1), baseline GA operators Sec. 6.1.  Where the paper
 * is silent (operators of the K-means GA, random streams, K-means features and
 * tie-breaks) the reading used is stated at each function.
 *
 * Deliberately slow and obvious: nested loops, no blocking, no fusion.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
 */
#include "pa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11, Sec. 3.2): a 4-word counter and a 2-word key go   */
/* through ten rounds; each round multiplies words 0 and 2 by two fixed odd   */
/* constants, keeps the 64-bit products' halves, permutes and xors with the   */
/* round key; the key is bumped by two Weyl constants between rounds.        */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void pao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream layout (the paper specifies no generator): key = the 64-bit seed,
 * counter = (c0, c1, c2, tag << 24 | block); block b holds words 4b..4b+3. */
uint32_t pao_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                  uint32_t idx) {
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {c0, c1, c2, (tag << 24) | (idx >> 2)};
  uint32_t out[4];
  pao_philox4x32_10(ctr, key, out);
  return out[idx & 3u];
}

/* Lemire's multiply-shift map of a 32-bit word onto [0, n), no rejection. */
uint32_t pao_bounded(uint32_t w, uint32_t n) {
  return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* An event of probability p happens when a 32-bit word is below floor(p*2^32). */
uint64_t pao_threshold(double p) {
  if (!(p >= 0.0)) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

/* ------------------------------------------------------------------------ */
/* Fitness: uplink sum spectral efficiency.                                  */
/* ------------------------------------------------------------------------ */

/* Checks that every row of a chromosome is a permutation of 0..K-1 and
 * builds the inverse: inv[j*K + s] = the user of cell j that sends pilot s. */
static int invert_rows(int L, int K, const uint8_t *chrom, int *inv) {
  for (int i = 0; i < L * K; ++i) inv[i] = -1;
  for (int j = 0; j < L; ++j)
    for (int k = 0; k < K; ++k) {
      int s = chrom[j * K + k];
      if (s >= K || inv[j * K + s] != -1) return -1;
      inv[j * K + s] = k;
    }
  return 0;
}

/*
 * SE of user k of cell i (Eq. 5): log2(1 + beta_iik^2 / sum_{j != i} beta_ijk^2),
 * where the interferer "user k of cell j" is read as the user of cell j that
 * reuses the pilot of user (i, k) (pilots are reused across cells, Sec. 3.1).
 *
 * Finite-M mode (the paper's Eq. 3 is garbled; this is the standard uplink
 * bound for maximum-ratio combining with MMSE estimates from tau-symbol
 * orthogonal pilots, pilot and data SNR rho, whose M -> infinity limit is
 * exactly Eq. 5):
 *   SINR = M tau rho^2 b^2 / ((1 + rho B_i)(1 + tau rho S) + M tau rho^2 I),
 *   S = sum_j beta_ijk' (own user included), I = sum_{j != i} beta_ijk'^2,
 *   B_i = sum_j sum_k beta_ijk (every user heard at BS i).
 */
/* Per-user SINR (want_sinr != 0) or SE = log2(1 + SINR) of one chromosome. */
static int user_terms(int32_t L, int32_t K, int32_t se_mode, double M, double rho,
                      const double *beta, const uint8_t *chrom, int want_sinr, double *se) {
  if (L < 1 || K < 1) return -1;
  int *inv = (int *)malloc(sizeof(int) * (size_t)L * K);
  if (!inv) return -2;
  if (invert_rows(L, K, chrom, inv) != 0) { free(inv); return -1; }
  const double tau = (double)K;
  for (int i = 0; i < L; ++i) {
    double B = 0.0;
    if (se_mode == PAO_SE_FINITE_M)
      for (int j = 0; j < L; ++j)
        for (int k = 0; k < K; ++k) B += beta[((size_t)i * L + j) * K + k];
    for (int k = 0; k < K; ++k) {
      int s = chrom[i * K + k];                 /* pilot of user (i, k) */
      double own = beta[((size_t)i * L + i) * K + k];
      double I = 0.0, S = 0.0;
      for (int j = 0; j < L; ++j) {
        int kj = inv[j * K + s];                /* user of cell j on pilot s */
        double g = beta[((size_t)i * L + j) * K + kj];
        S += g;
        if (j != i) I += g * g;
      }
      double sinr;
      if (se_mode == PAO_SE_FINITE_M) {
        double num = (double)M * tau * rho * rho * own * own;
        double den = (1.0 + rho * B) * (1.0 + tau * rho * S) + (double)M * tau * rho * rho * I;
        sinr = num / den;
      } else {
        sinr = own * own / I;
      }
      se[i * K + k] = want_sinr ? sinr : log2(1.0 + sinr);
    }
  }
  free(inv);
  return 0;
}

int pao_se_terms(int32_t L, int32_t K, int32_t se_mode, double M, double rho,
                 const double *beta, const uint8_t *chrom, double *se) {
  return user_terms(L, K, se_mode, M, rho, beta, chrom, 0, se);
}

int pao_sinr_terms(int32_t L, int32_t K, int32_t se_mode, double M, double rho,
                   const double *beta, const uint8_t *chrom, double *sinr) {
  return user_terms(L, K, se_mode, M, rho, beta, chrom, 1, sinr);
}

/*
 * Inter-cluster interference of Eq. 8 (Sec. 4.2), as read here: the printed
 * equation sums, over pairs of user clusters (c, c') that share a pilot, the
 * mean large-scale gain of c' at the BS of c over the mean gain of c at its own
 * BS, plus the same ratio with the roles swapped (the second numerator's
 * subscript is garbled in print: it must be c's users at the BS of c'). With
 * tau = K each cell's users sharing one pilot form a cluster of one user, so
 * the means are single gains, and summing both directions over every pair of
 * cells gives, per user (i, k) with pilot s,
 *     sum_{j != i} beta_i,j,k'(j) / beta_i,i,k,   k'(j) = user of cell j on s,
 * in first powers of beta (not squares). The pair (c, c) adds a constant and
 * is left out. The sum over all users is minimised.
 */
static int interference_ratio(int32_t L, int32_t K, const double *beta, const uint8_t *chrom,
                              double *out) {
  int *inv = (int *)malloc(sizeof(int) * (size_t)L * K);
  if (!inv) return -2;
  if (invert_rows(L, K, chrom, inv) != 0) { free(inv); return -1; }
  double total = 0.0;
  for (int i = 0; i < L; ++i)
    for (int k = 0; k < K; ++k) {
      int s = chrom[i * K + k];
      double own = beta[((size_t)i * L + i) * K + k];
      double I = 0.0;
      for (int j = 0; j < L; ++j)
        if (j != i) I += beta[((size_t)i * L + j) * K + inv[j * K + s]];
      total += I / own;
    }
  free(inv);
  *out = total;
  return 0;
}

/* Sum SE (Eq. 6), scaled by the share of the coherence interval left after
 * uplink training (Sec. 3): 1 - tau/T, or 1 when T == 0. */
/* objective 0: the sum over users of Eq. 7 times the pre-log; objective 1:
 * the smallest SINR of any user (the max-min SIR criterion the paper names
 * beside the sum, Sec. 2; SE is monotone in SINR, so it has the same optimum
 * as max-min SE); objective 2: minus the inter-cluster interference of Eq. 8
 * (interference_ratio; the GA maximises, the paper minimises; no pre-log,
 * independent of the SE mode). */
int pao_fitness_obj(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                    int32_t objective, const double *beta, const uint8_t *pop, int32_t n,
                    double *fit) {
  if (L < 1 || K < 1 || n < 0 || objective < 0 || objective > 2) return -1;
  if (objective == 2) {
    for (int c = 0; c < n; ++c) {
      double v = 0.0;
      int rc = interference_ratio(L, K, beta, pop + (size_t)c * L * K, &v);
      if (rc != 0) return rc;
      fit[c] = -v;
    }
    return 0;
  }
  double prelog = (T > 0) ? 1.0 - (double)K / (double)T : 1.0;
  double *se = (double *)malloc(sizeof(double) * (size_t)L * K);
  if (!se) return -2;
  for (int c = 0; c < n; ++c) {
    int rc = user_terms(L, K, se_mode, M, rho, beta, pop + (size_t)c * L * K, objective, se);
    if (rc != 0) { free(se); return rc; }
    double v = objective == 0 ? 0.0 : INFINITY;
    for (int i = 0; i < L; ++i)
      for (int k = 0; k < K; ++k) {
        if (objective == 0) v += se[i * K + k];
        else if (se[i * K + k] < v) v = se[i * K + k];
      }
    fit[c] = objective == 0 ? prelog * v : v;
  }
  free(se);
  return 0;
}

int pao_fitness(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                const double *beta, const uint8_t *pop, int32_t n, double *fit) {
  return pao_fitness_obj(L, K, T, se_mode, M, rho, 0, beta, pop, n, fit);
}

/* ------------------------------------------------------------------------ */
/* Ranking (elitism keeps the best candidates, Sec. 1 contribution 1).       */
/* a beats b when fit[a] > fit[b], or they are equal and a < b.  NaN ranks    */
/* below every number; among NaNs the lower index wins.                      */
/* ------------------------------------------------------------------------ */
static int beats(const double *fit, int a, int b) {
  double fa = fit[a], fb = fit[b];
  int na = isnan(fa), nb = isnan(fb);
  if (na || nb) {
    if (na && nb) return a < b;
    return nb;
  }
  if (fa > fb) return 1;
  if (fa < fb) return 0;
  return a < b;
}

int pao_rank(const double *fit, int32_t n, int32_t *order) {
  /* insertion sort: obviously correct, O(n^2) is fine for populations */
  for (int i = 0; i < n; ++i) {
    int v = i, pos = i;
    while (pos > 0 && beats(fit, v, order[pos - 1])) {
      order[pos] = order[pos - 1];
      --pos;
    }
    order[pos] = v;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* K-means seeding (Sec. 4.1: users are partitioned into spatial clusters,   */
/* and clustering initialises the population, Sec. 1 contribution 2).        */
/* Reading: features are each user's offset from its own BS in integer       */
/* millimetres; k = K clusters; farthest-point initial centroids; integer     */
/* Lloyd iterations (at most 100); then, per cell, users are matched to       */
/* cluster indices (= pilots) greedily by increasing distance.               */
/* ------------------------------------------------------------------------ */
#define KM_MAX_ITERS 100
#define KM_COORD_LIMIT (1ll << 23)

/* floor((2s + n) / (2n)): the mean s/n rounded half up, with floor division */
static int64_t rdiv(int64_t s, int64_t n) {
  int64_t num = 2 * s + n, den = 2 * n;
  int64_t q = num / den;
  if ((num % den != 0) && (num < 0)) q -= 1;
  return q;
}

static int64_t dist2(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  int64_t dx = ax - bx, dy = ay - by;
  return dx * dx + dy * dy;
}

int pao_kmeans_seed(int32_t L, int32_t K, const double *user_xy, const double *bs_xy,
                    uint8_t *seed_chrom, int32_t *centroids, int32_t *labels, int32_t *iters) {
  if (L < 1 || K < 1 || K > 255 || !user_xy || !bs_xy) return -1;
  const int n = L * K;
  int64_t *qx = (int64_t *)malloc(sizeof(int64_t) * n);
  int64_t *qy = (int64_t *)malloc(sizeof(int64_t) * n);
  int64_t *cx = (int64_t *)malloc(sizeof(int64_t) * K);
  int64_t *cy = (int64_t *)malloc(sizeof(int64_t) * K);
  int *lab = (int *)malloc(sizeof(int) * n);
  if (!qx || !qy || !cx || !cy || !lab) {
    free(qx); free(qy); free(cx); free(cy); free(lab);
    return -2;
  }
  int rc = 0;
  /* 1. features */
  for (int j = 0; j < L; ++j)
    for (int k = 0; k < K; ++k) {
      int u = j * K + k;
      double ox = 1000.0 * (user_xy[2 * u] - bs_xy[2 * j]);
      double oy = 1000.0 * (user_xy[2 * u + 1] - bs_xy[2 * j + 1]);
      if (!(fabs(ox) <= (double)KM_COORD_LIMIT) || !(fabs(oy) <= (double)KM_COORD_LIMIT)) rc = -1;
      else { qx[u] = llround(ox); qy[u] = llround(oy); }
    }
  if (rc != 0) goto done;
  /* 2. farthest-point initial centroids; ties to the lowest user index */
  for (int c = 0; c < K; ++c) {
    int best = -1;
    int64_t bestd = -1;
    for (int u = 0; u < n; ++u) {
      int64_t d;
      if (c == 0) {
        d = dist2(qx[u], qy[u], 0, 0);
      } else {
        d = INT64_MAX;
        for (int m = 0; m < c; ++m) {
          int64_t dm = dist2(qx[u], qy[u], cx[m], cy[m]);
          if (dm < d) d = dm;
        }
      }
      if (d > bestd) { bestd = d; best = u; }
    }
    cx[c] = qx[best];
    cy[c] = qy[best];
  }
  /* 3. Lloyd iterations: assign (ties to the lowest cluster), stop when no
   *    label changes, else move each non-empty centroid to its rounded mean */
  for (int u = 0; u < n; ++u) lab[u] = -1;
  int it = 0;
  for (it = 0; it < KM_MAX_ITERS; ++it) {
    int changed = 0;
    for (int u = 0; u < n; ++u) {
      int bc = 0;
      int64_t bd = dist2(qx[u], qy[u], cx[0], cy[0]);
      for (int c = 1; c < K; ++c) {
        int64_t d = dist2(qx[u], qy[u], cx[c], cy[c]);
        if (d < bd) { bd = d; bc = c; }
      }
      if (lab[u] != bc) { changed = 1; lab[u] = bc; }
    }
    if (!changed) break;
    for (int c = 0; c < K; ++c) {
      int64_t sx = 0, sy = 0, cnt = 0;
      for (int u = 0; u < n; ++u)
        if (lab[u] == c) { sx += qx[u]; sy += qy[u]; ++cnt; }
      if (cnt > 0) { cx[c] = rdiv(sx, cnt); cy[c] = rdiv(sy, cnt); }
    }
  }
  /* 4. per cell: visit the (user, cluster) pairs by increasing
   *    (distance, user, cluster) and give each free user a free cluster */
  for (int j = 0; j < L; ++j) {
    int *user_taken = (int *)calloc((size_t)K, sizeof(int));
    int *pilot_taken = (int *)calloc((size_t)K, sizeof(int));
    if (!user_taken || !pilot_taken) { free(user_taken); free(pilot_taken); rc = -2; goto done; }
    for (int step = 0; step < K; ++step) {
      int bk = -1, bp = -1;
      int64_t bd = INT64_MAX;
      for (int k = 0; k < K; ++k) {
        if (user_taken[k]) continue;
        for (int p = 0; p < K; ++p) {
          if (pilot_taken[p]) continue;
          int64_t d = dist2(qx[j * K + k], qy[j * K + k], cx[p], cy[p]);
          if (d < bd) { bd = d; bk = k; bp = p; }  /* strict: keeps lowest (k, p) */
        }
      }
      user_taken[bk] = 1;
      pilot_taken[bp] = 1;
      seed_chrom[j * K + bk] = (uint8_t)bp;
    }
    free(user_taken);
    free(pilot_taken);
  }
  if (centroids)
    for (int c = 0; c < K; ++c) { centroids[2 * c] = (int32_t)cx[c]; centroids[2 * c + 1] = (int32_t)cy[c]; }
  if (labels)
    for (int u = 0; u < n; ++u) labels[u] = lab[u];
  if (iters) *iters = it;
done:
  free(qx); free(qy); free(cx); free(cy); free(lab);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Genetic operators.                                                        */
/* ------------------------------------------------------------------------ */

/* Swap mutation of one chromosome: gene i = j*K + k (row-major) mutates when
 * its decision word is below thr; it then swaps pilots with user k' != k of
 * the same cell, drawn from the partner word.  Rows stay permutations. */
static void swap_mutate(int L, int K, uint8_t *chrom, uint64_t thr, uint64_t seed,
                        uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag_decide,
                        uint32_t tag_partner) {
  if (K < 2) return;
  for (int i = 0; i < L * K; ++i) {
    int j = i / K, k = i % K;
    uint32_t w = pao_word(seed, c0, c1, c2, tag_decide, (uint32_t)i);
    if ((uint64_t)w < thr) {
      uint32_t r = pao_bounded(pao_word(seed, c0, c1, c2, tag_partner, (uint32_t)i),
                               (uint32_t)(K - 1));
      int kp = (int)r + ((int)r >= k ? 1 : 0);
      uint8_t t = chrom[j * K + k];
      chrom[j * K + k] = chrom[j * K + kp];
      chrom[j * K + kp] = t;
    }
  }
}

/* Mutation codes of a child of the generation loop (the per-gene swap
 * mutation of the GA step; Sec. 6.1 mutates each gene with probability p_mut,
 * the paper fixes no random streams).  Each gene's decision is the event "its
 * 32-bit decision word is below thr(p_mut)", as for swap_mutate, but the
 * decision words are laid out bit-sliced: genes go in groups of 32 (group q
 * holds genes 32q .. 32q+31 of the row-major chromosome), and bit 31-k of the
 * decision word of gene 32q + b is bit b of word 32q + k of the MUT_DECIDE
 * stream (k = 0..31).  Distinct bits of independent uniform words are
 * independent uniform bits, so every decision word is uniform on [0, 2^32)
 * and independent of the others: the law of one word per gene.  The h-th
 * mutating gene of group q (h = 0, 1, .. in increasing gene order) draws its
 * partner from word 32q + h of the MUT_PARTNER stream: r = bounded(word,
 * K-1), partner k' = r + (r >= k).  codes[i] = k' + 1 for a mutating gene
 * i = j*K + k and 0 otherwise. */
static int mutation_codes_off(int32_t L, int32_t K, double p_mut, uint64_t seed, uint32_t slot,
                              uint32_t gen, uint32_t instance_id, uint32_t woff, uint8_t *codes);
int pao_mutation_codes(int32_t L, int32_t K, double p_mut, uint64_t seed, uint32_t slot,
                       uint32_t gen, uint32_t instance_id, uint8_t *codes) {
  return mutation_codes_off(L, K, p_mut, seed, slot, gen, instance_id, 0u, codes);
}

/* The same with every stream word index offset by woff (the island streams of
 * the island GA below use woff = island << 18: block bits 16..23 of the
 * counter). */
static int mutation_codes_off(int32_t L, int32_t K, double p_mut, uint64_t seed, uint32_t slot,
                              uint32_t gen, uint32_t instance_id, uint32_t woff, uint8_t *codes) {
  if (L < 1 || K < 1) return -1;
  const int LK = L * K;
  const uint64_t thr = pao_threshold(p_mut);
  memset(codes, 0, (size_t)LK);
  if (K < 2) return 0;
  for (int q = 0; 32 * q < LK; ++q) {
    uint32_t R[32];
    for (int k = 0; k < 32; ++k)
      R[k] = pao_word(seed, slot, gen, instance_id, PAO_TAG_MUT_DECIDE,
                      woff + (uint32_t)(32 * q + k));
    int h = 0;
    for (int b = 0; b < 32 && 32 * q + b < LK; ++b) {
      uint32_t w = 0;
      for (int k = 0; k < 32; ++k) w |= ((R[k] >> b) & 1u) << (31 - k);
      if ((uint64_t)w < thr) {
        const int i = 32 * q + b, k = i % K;
        uint32_t r = pao_bounded(pao_word(seed, slot, gen, instance_id, PAO_TAG_MUT_PARTNER,
                                          woff + (uint32_t)(32 * q + h)),
                                 (uint32_t)(K - 1));
        codes[i] = (uint8_t)((int)r + ((int)r >= k ? 1 : 0) + 1);
        ++h;
      }
    }
  }
  return 0;
}

/* Applies mutation codes to a chromosome: genes in increasing row-major
 * order, each mutating gene swapping pilots with its partner in the current
 * row.  Rows stay permutations. */
static void apply_codes(int L, int K, uint8_t *chrom, const uint8_t *codes) {
  for (int i = 0; i < L * K; ++i) {
    if (!codes[i]) continue;
    int j = i / K, k = i % K, kp = codes[i] - 1;
    uint8_t t = chrom[j * K + k];
    chrom[j * K + k] = chrom[j * K + kp];
    chrom[j * K + kp] = t;
  }
}

/* Initial population.  Individual 0 is the K-means seed, individuals
 * 1..n_km-1 are the seed after swap mutation at rate p_init, and the rest are
 * uniformly random rows (Fisher-Yates from the identity), i.e. the random
 * initialisation of the conventional GA (Alg. 1, Sec. 6.1). */
int pao_init_pop(int32_t L, int32_t K, int32_t N, double kmeans_frac, double p_init,
                 uint64_t seed, uint32_t instance_id, const uint8_t *seed_chrom, uint8_t *pop) {
  if (L < 1 || K < 1 || N < 1) return -1;
  int n_km = 0;
  if (kmeans_frac > 0.0) {
    n_km = (int)floor(kmeans_frac * (double)N + 0.5);
    if (n_km < 1) n_km = 1;
    if (n_km > N) n_km = N;
    if (!seed_chrom) return -1;
  }
  const uint32_t c1 = 0xFFFFFFFFu;
  const uint64_t thr = pao_threshold(p_init);
  for (int n = 0; n < N; ++n) {
    uint8_t *chrom = pop + (size_t)n * L * K;
    if (n < n_km) {
      memcpy(chrom, seed_chrom, (size_t)L * K);
      if (n >= 1)
        swap_mutate(L, K, chrom, thr, seed, (uint32_t)n, c1, instance_id, PAO_TAG_INIT_DECIDE,
                    PAO_TAG_INIT_PARTNER);
    } else {
      for (int j = 0; j < L; ++j) {
        uint8_t *row = chrom + j * K;
        for (int k = 0; k < K; ++k) row[k] = (uint8_t)k;
        for (int k = K - 1; k >= 1; --k) {
          uint32_t w = pao_word(seed, (uint32_t)n, c1, instance_id, PAO_TAG_INIT_SHUFFLE,
                                (uint32_t)(j * K + k));
          int r = (int)pao_bounded(w, (uint32_t)(k + 1));
          uint8_t t = row[k];
          row[k] = row[r];
          row[r] = t;
        }
      }
    }
  }
  return 0;
}

/* One generation (Alg. 1 loop body with a single panmictic population):
 *  - elitism: slots 0..E-1 get the E best chromosomes in rank order;
 *  - children fill slots E, E+1, ... in pairs (a, a+1); each pair draws six
 *    SELECT words keyed by slot a: two binary tournaments pick the parents,
 *    word 4 decides single-point crossover (probability p_cross, Sec. 6.1),
 *    applied on the cell axis so rows stay permutations, word 5 the cut;
 *  - each child is swap-mutated with per-gene probability p_mut, keyed by its
 *    own slot (pao_mutation_codes).  If N - E is odd the last pair keeps
 *    child a only. */
int pao_ga_step(int32_t L, int32_t K, int32_t N, int32_t E, double p_cross, double p_mut,
                uint64_t seed, uint32_t instance_id, uint32_t gen, const uint8_t *pop_in,
                const double *fit_in, uint8_t *pop_out) {
  if (L < 1 || K < 1 || N < 1 || E < 0 || E > N) return -1;
  const size_t G = (size_t)L * K;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
  if (!order) return -2;
  pao_rank(fit_in, N, order);
  for (int e = 0; e < E; ++e) memcpy(pop_out + e * G, pop_in + (size_t)order[e] * G, G);
  free(order);

  const uint64_t thr_c = pao_threshold(p_cross);
  uint8_t *codes = (uint8_t *)malloc(G);
  if (!codes) return -2;
  for (int a = E; a < N; a += 2) {
    int b = a + 1;
    uint32_t w[6];
    for (int i = 0; i < 6; ++i)
      w[i] = pao_word(seed, (uint32_t)a, gen, instance_id, PAO_TAG_SELECT, (uint32_t)i);
    int u0 = (int)pao_bounded(w[0], (uint32_t)N), v0 = (int)pao_bounded(w[1], (uint32_t)N);
    int u1 = (int)pao_bounded(w[2], (uint32_t)N), v1 = (int)pao_bounded(w[3], (uint32_t)N);
    int p1 = beats(fit_in, v0, u0) ? v0 : u0;
    int p2 = beats(fit_in, v1, u1) ? v1 : u1;
    uint8_t *ca = pop_out + (size_t)a * G;
    uint8_t *cb = (b < N) ? pop_out + (size_t)b * G : NULL;
    const uint8_t *P1 = pop_in + (size_t)p1 * G, *P2 = pop_in + (size_t)p2 * G;
    if (L >= 2 && (uint64_t)w[4] < thr_c) {
      int cut = 1 + (int)pao_bounded(w[5], (uint32_t)(L - 1));
      for (int j = 0; j < L; ++j) {
        const uint8_t *ra = (j < cut) ? P1 : P2;
        const uint8_t *rb = (j < cut) ? P2 : P1;
        memcpy(ca + j * K, ra + j * K, (size_t)K);
        if (cb) memcpy(cb + j * K, rb + j * K, (size_t)K);
      }
    } else {
      memcpy(ca, P1, G);
      if (cb) memcpy(cb, P2, G);
    }
    pao_mutation_codes(L, K, p_mut, seed, (uint32_t)a, gen, instance_id, codes);
    apply_codes(L, K, ca, codes);
    if (cb) {
      pao_mutation_codes(L, K, p_mut, seed, (uint32_t)b, gen, instance_id, codes);
      apply_codes(L, K, cb, codes);
    }
  }
  free(codes);
  return 0;
}

static double max_fit(const double *fit, int n) {
  int best = 0;
  for (int i = 1; i < n; ++i)
    if (beats(fit, i, best)) best = i;
  return fit[best];
}

/* The sequential K-means GA (Alg. 1) with a fixed number of generations:
 * seed, initialise, then per generation evaluate, select and evolve; return
 * the best assignment of the last population. */
int pao_solve(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
              const double *beta, const double *user_xy, const double *bs_xy, int32_t N,
              int32_t gens, int32_t E, double p_cross, double p_mut, double kmeans_frac,
              double p_init, uint64_t seed, uint32_t instance_id, uint8_t *best,
              double *best_fit, double *trace, uint8_t *final_pop) {
  if (L < 1 || K < 1 || N < 1 || gens < 0 || E < 0 || E > N) return -1;
  const size_t G = (size_t)L * K;
  uint8_t *popA = (uint8_t *)malloc(G * N), *popB = (uint8_t *)malloc(G * N);
  double *fit = (double *)malloc(sizeof(double) * N);
  uint8_t *seed_chrom = (uint8_t *)malloc(G);
  int rc = 0;
  if (!popA || !popB || !fit || !seed_chrom) { rc = -2; goto out; }
  if (kmeans_frac > 0.0) {
    rc = pao_kmeans_seed(L, K, user_xy, bs_xy, seed_chrom, NULL, NULL, NULL);
    if (rc) goto out;
  }
  rc = pao_init_pop(L, K, N, kmeans_frac, p_init, seed, instance_id,
                    kmeans_frac > 0.0 ? seed_chrom : NULL, popA);
  if (rc) goto out;
  rc = pao_fitness(L, K, T, se_mode, M, rho, beta, popA, N, fit);
  if (rc) goto out;
  for (int g = 0; g < gens; ++g) {
    if (trace) trace[g] = max_fit(fit, N);
    rc = pao_ga_step(L, K, N, E, p_cross, p_mut, seed, instance_id, (uint32_t)g, popA, fit, popB);
    if (rc) goto out;
    uint8_t *t = popA; popA = popB; popB = t;
    rc = pao_fitness(L, K, T, se_mode, M, rho, beta, popA, N, fit);
    if (rc) goto out;
  }
  if (trace) trace[gens] = max_fit(fit, N);
  {
    int b = 0;
    for (int i = 1; i < N; ++i)
      if (beats(fit, i, b)) b = i;
    memcpy(best, popA + (size_t)b * G, G);
    *best_fit = fit[b];
  }
  if (final_pop) memcpy(final_pop, popA, G * N);
out:
  free(popA); free(popB); free(fit); free(seed_chrom);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* The parallel K-means GA (PK-means GA, Alg. 2, Sec. 4.3): the population is */
/* partitioned by K-means into C clusters (islands) that evolve on their own;  */
/* K-means is applied again every few generations (three in Sec. 6.1).  The   */
/* paper fixes neither the feature space nor the per-island operators; the    */
/* reading here:                                                              */
/*  - a chromosome is the point (g_0, .., g_{LK-1}) of Z^{LK} (its pilot       */
/*    indices), squared Euclidean distance in integers;                       */
/*  - farthest-point start: centroid 0 is the best-ranked chromosome, centroid */
/*    m the chromosome farthest from centroids 0..m-1 (distance to the nearest */
/*    one; ties to the lowest index); then Lloyd iterations (assign to the     */
/*    nearest centroid, ties to the lowest cluster; centroid = per-gene        */
/*    rounded mean floor((2 s + n) / (2 n)); an empty cluster keeps its        */
/*    centroid) until no label changes or max_iters;                          */
/*  - island c holds the positions labelled c (increasing order) and keeps them*/
/*    until the next clustering: its children take its positions;            */
/*  - per island, the GA step of pao_ga_step restricted to the island: E_c =  */
/*    0 if E = 0, else min(n_c, max(1, floor(E n_c / N + 1/2))) elites (the    */
/*    island's best in rank order) in its first E_c positions; children in    */
/*    pairs over the following positions (a, b consecutive positions of the   */
/*    island), tournament candidates drawn among the island's members;       */
/*  - the island's random streams are those of pao_ga_step (keyed by the      */
/*    global slot of the pair's first child, or of the child) with the island */
/*    index in bits 16..23 of the block counter, so with C = 1 the island GA   */
/*    is the panmictic GA bit for bit.                                         */
/* ------------------------------------------------------------------------ */

static int64_t chrom_dist2(const uint8_t *a, const uint8_t *b, int n) {
  int64_t d = 0;
  for (int i = 0; i < n; ++i) {
    int64_t t = (int64_t)a[i] - (int64_t)b[i];
    d += t * t;
  }
  return d;
}

int pao_pop_kmeans(int32_t L, int32_t K, int32_t N, int32_t C, const uint8_t *pop,
                   const double *fit, int32_t max_iters, int32_t *labels, uint8_t *centroids,
                   int32_t *iters) {
  if (L < 1 || K < 1 || N < 1 || C < 1 || C > N || max_iters < 1) return -1;
  const int G = L * K;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
  int64_t *sums = (int64_t *)malloc(sizeof(int64_t) * (size_t)C * G);
  int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * C);
  uint8_t *cent = (uint8_t *)malloc((size_t)C * G);
  int rc = 0;
  if (!order || !sums || !cnt || !cent) { rc = -2; goto done; }
  pao_rank(fit, N, order);
  memcpy(cent, pop + (size_t)order[0] * G, (size_t)G);
  for (int m = 1; m < C; ++m) {
    int far = 0;
    int64_t far_d = -1;
    for (int n = 0; n < N; ++n) {
      int64_t dmin = -1;
      for (int c = 0; c < m; ++c) {
        int64_t d = chrom_dist2(pop + (size_t)n * G, cent + (size_t)c * G, G);
        if (dmin < 0 || d < dmin) dmin = d;
      }
      if (dmin > far_d) { far_d = dmin; far = n; }
    }
    memcpy(cent + (size_t)m * G, pop + (size_t)far * G, (size_t)G);
  }
  for (int n = 0; n < N; ++n) labels[n] = -1;
  int it = 0;
  for (; it < max_iters; ++it) {
    int changed = 0;
    for (int n = 0; n < N; ++n) {
      int best = 0;
      int64_t bd = -1;
      for (int c = 0; c < C; ++c) {
        int64_t d = chrom_dist2(pop + (size_t)n * G, cent + (size_t)c * G, G);
        if (bd < 0 || d < bd) { bd = d; best = c; }
      }
      if (labels[n] != best) { labels[n] = best; changed = 1; }
    }
    if (!changed) break;
    memset(sums, 0, sizeof(int64_t) * (size_t)C * G);
    memset(cnt, 0, sizeof(int32_t) * C);
    for (int n = 0; n < N; ++n) {
      ++cnt[labels[n]];
      for (int i = 0; i < G; ++i) sums[(size_t)labels[n] * G + i] += pop[(size_t)n * G + i];
    }
    for (int c = 0; c < C; ++c) {
      if (cnt[c] == 0) continue;
      for (int i = 0; i < G; ++i) {
        int64_t s2 = 2 * sums[(size_t)c * G + i] + cnt[c];
        cent[(size_t)c * G + i] = (uint8_t)(s2 / (2 * (int64_t)cnt[c]));  /* s >= 0: floor */
      }
    }
  }
  if (centroids) memcpy(centroids, cent, (size_t)C * G);
  if (iters) *iters = it;
done:
  free(order); free(sums); free(cnt); free(cent);
  return rc;
}

static int island_elites(int E, int N, int n) {
  if (E == 0 || n == 0) return 0;
  int e = (int)((2 * (int64_t)E * n + N) / (2 * (int64_t)N));
  if (e < 1) e = 1;
  return e > n ? n : e;
}

int pao_island_step(int32_t L, int32_t K, int32_t N, int32_t E, int32_t C,
                    const int32_t *labels, double p_cross, double p_mut, uint64_t seed,
                    uint32_t instance_id, uint32_t gen, const uint8_t *pop_in,
                    const double *fit_in, uint8_t *pop_out) {
  if (L < 1 || K < 1 || N < 1 || E < 0 || E > N || C < 1 || C > 255) return -1;
  const size_t G = (size_t)L * K;
  int32_t *M = (int32_t *)malloc(sizeof(int32_t) * N);
  double *sub = (double *)malloc(sizeof(double) * N);
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
  uint8_t *codes = (uint8_t *)malloc(G);
  if (!M || !sub || !order || !codes) { free(M); free(sub); free(order); free(codes); return -2; }
  const uint64_t thr_c = pao_threshold(p_cross);
  for (int c = 0; c < C; ++c) {
    int n = 0;
    for (int i = 0; i < N; ++i)
      if (labels[i] == c) M[n++] = i;
    if (n == 0) continue;
    const uint32_t woff = (uint32_t)c << 18;
    /* the island's members ranked: order[] indexes M[] */
    for (int t = 0; t < n; ++t) sub[t] = fit_in[M[t]];
    pao_rank(sub, n, order);
    const int Ec = island_elites(E, N, n);
    for (int e = 0; e < Ec; ++e)
      memcpy(pop_out + (size_t)M[e] * G, pop_in + (size_t)M[order[e]] * G, G);
    for (int t = Ec; t < n; t += 2) {
      const int a = M[t];
      const int has_b = t + 1 < n;
      const int b = has_b ? M[t + 1] : -1;
      uint32_t w[6];
      for (int i = 0; i < 6; ++i)
        w[i] = pao_word(seed, (uint32_t)a, gen, instance_id, PAO_TAG_SELECT, woff + (uint32_t)i);
      int u0 = M[pao_bounded(w[0], (uint32_t)n)], v0 = M[pao_bounded(w[1], (uint32_t)n)];
      int u1 = M[pao_bounded(w[2], (uint32_t)n)], v1 = M[pao_bounded(w[3], (uint32_t)n)];
      int p1 = beats(fit_in, v0, u0) ? v0 : u0;
      int p2 = beats(fit_in, v1, u1) ? v1 : u1;
      uint8_t *ca = pop_out + (size_t)a * G;
      uint8_t *cb = has_b ? pop_out + (size_t)b * G : NULL;
      const uint8_t *P1 = pop_in + (size_t)p1 * G, *P2 = pop_in + (size_t)p2 * G;
      if (L >= 2 && (uint64_t)w[4] < thr_c) {
        int cut = 1 + (int)pao_bounded(w[5], (uint32_t)(L - 1));
        for (int j = 0; j < L; ++j) {
          memcpy(ca + j * K, ((j < cut) ? P1 : P2) + j * K, (size_t)K);
          if (cb) memcpy(cb + j * K, ((j < cut) ? P2 : P1) + j * K, (size_t)K);
        }
      } else {
        memcpy(ca, P1, G);
        if (cb) memcpy(cb, P2, G);
      }
      mutation_codes_off(L, K, p_mut, seed, (uint32_t)a, gen, instance_id, woff, codes);
      apply_codes(L, K, ca, codes);
      if (cb) {
        mutation_codes_off(L, K, p_mut, seed, (uint32_t)b, gen, instance_id, woff, codes);
        apply_codes(L, K, cb, codes);
      }
    }
  }
  free(M); free(sub); free(order); free(codes);
  return 0;
}

int pao_island_solve(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                     const double *beta, const double *user_xy, const double *bs_xy, int32_t N,
                     int32_t gens, int32_t E, double p_cross, double p_mut, double kmeans_frac,
                     double p_init, uint64_t seed, uint32_t instance_id, int32_t C,
                     int32_t recluster_every, int32_t max_iters, uint8_t *best, double *best_fit,
                     double *trace, uint8_t *final_pop, int32_t *final_labels) {
  if (L < 1 || K < 1 || N < 1 || gens < 0 || E < 0 || E > N || C < 1 || C > N ||
      recluster_every < 0)
    return -1;
  const size_t G = (size_t)L * K;
  uint8_t *popA = (uint8_t *)malloc(G * N), *popB = (uint8_t *)malloc(G * N);
  double *fit = (double *)malloc(sizeof(double) * N);
  uint8_t *seed_chrom = (uint8_t *)malloc(G);
  int32_t *labels = (int32_t *)calloc((size_t)N, sizeof(int32_t));
  int rc = 0;
  if (!popA || !popB || !fit || !seed_chrom || !labels) { rc = -2; goto out; }
  if (kmeans_frac > 0.0) {
    rc = pao_kmeans_seed(L, K, user_xy, bs_xy, seed_chrom, NULL, NULL, NULL);
    if (rc) goto out;
  }
  rc = pao_init_pop(L, K, N, kmeans_frac, p_init, seed, instance_id,
                    kmeans_frac > 0.0 ? seed_chrom : NULL, popA);
  if (rc) goto out;
  rc = pao_fitness(L, K, T, se_mode, M, rho, beta, popA, N, fit);
  if (rc) goto out;
  for (int g = 0; g < gens; ++g) {
    if (trace) trace[g] = max_fit(fit, N);
    /* Alg. 2: apply K-means (every recluster_every generations; 0 = only at
       the start) */
    if (C > 1 && (g == 0 || (recluster_every > 0 && g % recluster_every == 0))) {
      rc = pao_pop_kmeans(L, K, N, C, popA, fit, max_iters, labels, NULL, NULL);
      if (rc) goto out;
    }
    rc = pao_island_step(L, K, N, E, C, labels, p_cross, p_mut, seed, instance_id,
                         (uint32_t)g, popA, fit, popB);
    if (rc) goto out;
    uint8_t *t = popA; popA = popB; popB = t;
    rc = pao_fitness(L, K, T, se_mode, M, rho, beta, popA, N, fit);
    if (rc) goto out;
  }
  if (trace) trace[gens] = max_fit(fit, N);
  {
    int b = 0;
    for (int i = 1; i < N; ++i)
      if (beats(fit, i, b)) b = i;
    memcpy(best, popA + (size_t)b * G, G);
    *best_fit = fit[b];
  }
  if (final_pop) memcpy(final_pop, popA, G * N);
  if (final_labels) memcpy(final_labels, labels, sizeof(int32_t) * N);
out:
  free(popA); free(popB); free(fit); free(seed_chrom); free(labels);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive pilot assignment (EX-PA, Sec. 6.2; K!^(L-1) classes, Sec. 3.3) */
/* Relabelling the pilots the same way in every cell leaves Eq. 7 unchanged, */
/* so row 0 is fixed to the identity and rows 1..L-1 run over all K! orders. */
/* ------------------------------------------------------------------------ */
static int next_permutation(uint8_t *a, int n) {
  int i = n - 2;
  while (i >= 0 && a[i] >= a[i + 1]) --i;
  if (i < 0) { /* last order: wrap back to ascending */
    for (int l = 0, r = n - 1; l < r; ++l, --r) { uint8_t t = a[l]; a[l] = a[r]; a[r] = t; }
    return 0;
  }
  int j = n - 1;
  while (a[j] <= a[i]) --j;
  uint8_t t = a[i]; a[i] = a[j]; a[j] = t;
  for (int l = i + 1, r = n - 1; l < r; ++l, --r) { t = a[l]; a[l] = a[r]; a[r] = t; }
  return 1;
}

int pao_bruteforce(int32_t L, int32_t K, int32_t T, int32_t se_mode, double M, double rho,
                   const double *beta, uint8_t *best, double *best_fit, int64_t *count) {
  if (L < 1 || K < 1 || K > 12) return -1;
  const size_t G = (size_t)L * K;
  uint8_t *chrom = (uint8_t *)malloc(G);
  if (!chrom) return -2;
  for (int j = 0; j < L; ++j)
    for (int k = 0; k < K; ++k) chrom[j * K + k] = (uint8_t)k;
  double bf = -INFINITY;
  int64_t cnt = 0;
  for (;;) {
    double f;
    int rc = pao_fitness(L, K, T, se_mode, M, rho, beta, chrom, 1, &f);
    if (rc) { free(chrom); return rc; }
    ++cnt;
    if (f > bf) { bf = f; memcpy(best, chrom, G); }
    /* odometer over rows L-1 .. 1 */
    int j = L - 1;
    while (j >= 1) {
      if (next_permutation(chrom + j * K, K)) break;
      /* wrapped: next_permutation left the row sorted ascending (identity) */
      --j;
    }
    if (j < 1) break;
  }
  *best_fit = bf;
  if (count) *count = cnt;
  free(chrom);
  return 0;
}
