/*
 * Random walk on the flip graph of <M,K,N> matrix multiplication schemes over
 * GF(2) (Kauers and Moosbauer, "Flip graphs for matrix multiplication", ISSAC
 * 2023), used to find bilinear algorithms of a given rank.
 *
 * A scheme is a list of rank-one terms u_r (x) v_r (x) w_r, with u_r a subset of
 * the M*K blocks of A, v_r of the K*N blocks of B and w_r of the M*N blocks of
 * C (bit masks, row-wise block order as in Section 2.2 of the paper), whose
 * sum over GF(2) is the matrix multiplication tensor: block product
 * A_ab B_bc contributes to C_ac.  The walk starts from the classical scheme
 * (rank M*K*N) and applies:
 *   flip:      two terms sharing a factor, u (x) v1 (x) w1 + u (x) v2 (x) w2
 *              = u (x) (v1 + v2) (x) w1 + u (x) v2 (x) (w1 + w2)  (mod 2),
 *              and likewise for a shared v or w;
 *   reduction: a term with an empty factor is dropped; two terms sharing two
 *              factors merge into one (rank - 1);
 *   plus:      after `plateau` flips without a reduction the scheme is
 *              enlarged by one term, t1 + t2 = t1' + t2a + t2b with
 *              t2a sharing a factor with t1 (rank + 1), which opens new flips.
 * Every scheme it prints is checked against the tensor over GF(2) first.
 *
 * The same walk over the integers ('z' mode) keeps every coefficient in
 * {-1, 0, 1}: a flip u (x) v1 (x) w1 + u (x) v2 (x) w2 =
 * u (x) (v1 + s v2) (x) w1 + u (x) v2 (x) (w2 - s w1), s = +-1, is an identity
 * over Z, so every scheme met is an exact algorithm and needs no lifting;
 * moves that would leave {-1, 0, 1} are not taken.  Terms are kept
 * normalised (first non-zero of u and of v positive, signs moved into w), so
 * factors equal up to sign compare equal.
 *
 * usage: search M K N target seed max_flips plateau count [z]
 * prints up to `count` schemes of rank <= target: over GF(2) the first one
 * reached and then every 1000th flip's neighbour at that rank; over Z one per
 * walk, restarting from the classical scheme after each hit.  Each scheme is
 * one line
 *   GF(2):  "R u_0 v_0 w_0 u_1 ..." (hexadecimal masks)
 *   z:      "R u_0 v_0 w_0 u_1 ..." (one character per coefficient: n = -1, 0, 1)
 * Build: gcc -O2 -o search search.c
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXR 160

static int M, K, N;
static uint32_t U[MAXR], V[MAXR], W[MAXR];
static int R;

/* xorshift64*: the walk's only source of randomness, seeded by the caller */
static uint64_t rng_state;
static uint64_t rnd(void) {
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 2685821657736338717ULL;
}
static int rnd_below(int n) { return (int)(rnd() % (uint64_t)n); }

static void classical(void) {
  R = 0;
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < K; ++b)
      for (int c = 0; c < N; ++c) {
        U[R] = 1u << (a * K + b);
        V[R] = 1u << (b * N + c);
        W[R] = 1u << (a * N + c);
        ++R;
      }
}

/* Sum of the terms over GF(2) equals the tensor. */
static int check(void) {
  for (int i = 0; i < M * K; ++i)
    for (int j = 0; j < K * N; ++j)
      for (int k = 0; k < M * N; ++k) {
        int s = 0;
        for (int r = 0; r < R; ++r) s ^= (int)(((U[r] >> i) & (V[r] >> j) & (W[r] >> k)) & 1u);
        const int ia = i / K, ib = i % K, jb = j / N, jc = j % N, ka = k / N, kc = k % N;
        const int t = (ib == jb && jc == kc && ia == ka) ? 1 : 0;
        if (s != t) return 0;
      }
  return 1;
}

static void drop(int r) {
  --R;
  U[r] = U[R];
  V[r] = V[R];
  W[r] = W[R];
}

/* Applies reductions until none is left; returns how many terms went. */
static int reduce(void) {
  int removed = 0, again = 1;
  while (again) {
    again = 0;
    for (int r = 0; r < R; ++r)
      if (!U[r] || !V[r] || !W[r]) {
        drop(r);
        ++removed;
        again = 1;
        break;
      }
    if (again) continue;
    for (int i = 0; i < R && !again; ++i)
      for (int j = i + 1; j < R && !again; ++j) {
        if (U[i] == U[j] && V[i] == V[j]) W[i] ^= W[j];
        else if (U[i] == U[j] && W[i] == W[j]) V[i] ^= V[j];
        else if (V[i] == V[j] && W[i] == W[j]) U[i] ^= U[j];
        else continue;
        drop(j);
        ++removed;
        again = 1;
      }
  }
  return removed;
}

/* One random flip; 0 if the chosen term shares no factor with another. */
static int flip(void) {
  const int i = rnd_below(R), slot = rnd_below(3);
  int cand[MAXR], nc = 0;
  for (int j = 0; j < R; ++j) {
    if (j == i) continue;
    if ((slot == 0 && U[j] == U[i]) || (slot == 1 && V[j] == V[i]) || (slot == 2 && W[j] == W[i])) cand[nc++] = j;
  }
  if (!nc) return 0;
  const int j = cand[rnd_below(nc)];
  /* shared factor in `slot`: term i takes the sum of one of the other two
     factors, term j the sum of the remaining one */
  if (slot == 0) {
    V[i] ^= V[j];
    W[j] ^= W[i];
  } else if (slot == 1) {
    U[i] ^= U[j];
    W[j] ^= W[i];
  } else {
    U[i] ^= U[j];
    V[j] ^= V[i];
  }
  return 1;
}

/* Plus transition: terms t1 = a (x) b (x) c and t2 = a' (x) b' (x) c' become
   t1, a' (x) b (x) c' and a' (x) (b + b') (x) c' (mod 2 the last two sum to t2). */
static void plus(void) {
  if (R + 1 >= MAXR || R < 2) return;
  const int i = rnd_below(R);
  int j = rnd_below(R - 1);
  if (j >= i) ++j;
  U[R] = U[j];
  V[R] = V[j] ^ V[i];
  W[R] = W[j];
  V[j] = V[i];
  ++R;
}

/* ---- the walk over the integers -------------------------------------- */

typedef signed char i8;
static i8 ZU[MAXR][32], ZV[MAXR][32], ZW[MAXR][32];
static int MK, KN, MN;

static void zclassical(void) {
  R = 0;
  memset(ZU, 0, sizeof(ZU));
  memset(ZV, 0, sizeof(ZV));
  memset(ZW, 0, sizeof(ZW));
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < K; ++b)
      for (int c = 0; c < N; ++c) {
        ZU[R][a * K + b] = 1;
        ZV[R][b * N + c] = 1;
        ZW[R][a * N + c] = 1;
        ++R;
      }
}

static int zzero(const i8* x, int n) {
  for (int i = 0; i < n; ++i)
    if (x[i]) return 0;
  return 1;
}
static int zeq(const i8* x, const i8* y, int n) { return memcmp(x, y, (size_t)n) == 0; }
static int zneg_eq(const i8* x, const i8* y, int n) {
  for (int i = 0; i < n; ++i)
    if (x[i] != -y[i]) return 0;
  return 1;
}
static void zneg(i8* x, int n) {
  for (int i = 0; i < n; ++i) x[i] = (i8)-x[i];
}
/* x += s y if every result stays in {-1, 0, 1}; returns 0 (x unchanged) else */
static int zaxpy(i8* x, int s, const i8* y, int n) {
  i8 t[32];
  for (int i = 0; i < n; ++i) {
    const int v = x[i] + s * y[i];
    if (v < -1 || v > 1) return 0;
    t[i] = (i8)v;
  }
  memcpy(x, t, (size_t)n);
  return 1;
}
static void znorm(int r) {
  for (int i = 0; i < MK; ++i)
    if (ZU[r][i]) {
      if (ZU[r][i] < 0) {
        zneg(ZU[r], MK);
        zneg(ZW[r], MN);
      }
      break;
    }
  for (int j = 0; j < KN; ++j)
    if (ZV[r][j]) {
      if (ZV[r][j] < 0) {
        zneg(ZV[r], KN);
        zneg(ZW[r], MN);
      }
      break;
    }
}
static void zdrop(int r) {
  --R;
  memcpy(ZU[r], ZU[R], 32);
  memcpy(ZV[r], ZV[R], 32);
  memcpy(ZW[r], ZW[R], 32);
}

static int zcheck(void) {
  for (int i = 0; i < MK; ++i)
    for (int j = 0; j < KN; ++j)
      for (int k = 0; k < MN; ++k) {
        int s = 0;
        for (int r = 0; r < R; ++r) s += ZU[r][i] * ZV[r][j] * ZW[r][k];
        const int ia = i / K, ib = i % K, jb = j / N, jc = j % N, ka = k / N, kc = k % N;
        if (s != ((ib == jb && jc == kc && ia == ka) ? 1 : 0)) return 0;
      }
  return 1;
}

static int zreduce(void) {
  int removed = 0, again = 1;
  while (again) {
    again = 0;
    for (int r = 0; r < R; ++r)
      if (zzero(ZU[r], MK) || zzero(ZV[r], KN) || zzero(ZW[r], MN)) {
        zdrop(r);
        ++removed;
        again = 1;
        break;
      }
    if (again) continue;
    for (int i = 0; i < R && !again; ++i)
      for (int j = i + 1; j < R && !again; ++j) {
        const int eu = zeq(ZU[i], ZU[j], MK), ev = zeq(ZV[i], ZV[j], KN);
        const int ew = zeq(ZW[i], ZW[j], MN) ? 1 : zneg_eq(ZW[i], ZW[j], MN) ? -1 : 0;
        int merged = 0;
        if (eu && ev) merged = zaxpy(ZW[i], 1, ZW[j], MN);
        else if (eu && ew) merged = zaxpy(ZV[i], ew, ZV[j], KN);
        else if (ev && ew) merged = zaxpy(ZU[i], ew, ZU[j], MK);
        if (!merged) continue;
        zdrop(j);
        znorm(i);
        ++removed;
        again = 1;
      }
  }
  return removed;
}

static int zflip(void) {
  const int i = rnd_below(R), slot = rnd_below(3);
  int cand[MAXR], sg[MAXR], nc = 0;
  for (int j = 0; j < R; ++j) {
    if (j == i) continue;
    if (slot == 0 && zeq(ZU[j], ZU[i], MK)) sg[nc] = 1, cand[nc++] = j;
    else if (slot == 1 && zeq(ZV[j], ZV[i], KN)) sg[nc] = 1, cand[nc++] = j;
    else if (slot == 2 && zeq(ZW[j], ZW[i], MN)) sg[nc] = 1, cand[nc++] = j;
    else if (slot == 2 && zneg_eq(ZW[j], ZW[i], MN)) sg[nc] = -1, cand[nc++] = j;
  }
  if (!nc) return 0;
  const int q = rnd_below(nc), j = cand[q];
  const int s = (rnd() & 1) ? 1 : -1;
  i8 a[32], b[32];
  if (slot == 0) {
    /* u (x) vi (x) wi + u (x) vj (x) wj = u (x) (vi + s vj) (x) wi + u (x) vj (x) (wj - s wi) */
    memcpy(a, ZV[i], 32);
    memcpy(b, ZW[j], 32);
    if (!zaxpy(a, s, ZV[j], KN) || !zaxpy(b, -s, ZW[i], MN)) return 0;
    memcpy(ZV[i], a, 32);
    memcpy(ZW[j], b, 32);
  } else if (slot == 1) {
    /* ui (x) v (x) wi + uj (x) v (x) wj = (ui + s uj) (x) v (x) wi + uj (x) v (x) (wj - s wi) */
    memcpy(a, ZU[i], 32);
    memcpy(b, ZW[j], 32);
    if (!zaxpy(a, s, ZU[j], MK) || !zaxpy(b, -s, ZW[i], MN)) return 0;
    memcpy(ZU[i], a, 32);
    memcpy(ZW[j], b, 32);
  } else {
    /* wj = g wi: ui (x) vi (x) w + (g uj) (x) vj (x) w
       = (ui + s g uj) (x) vi (x) w + (g uj) (x) (vj - s vi) (x) w */
    const int g = sg[q];
    memcpy(a, ZU[i], 32);
    memcpy(b, ZV[j], 32);
    if (!zaxpy(a, s * g, ZU[j], MK) || !zaxpy(b, -s, ZV[i], KN)) return 0;
    memcpy(ZU[i], a, 32);
    memcpy(ZV[j], b, 32);
  }
  znorm(i);
  znorm(j);
  return 1;
}

/* plus: tj = a (x) b (x) c becomes a (x) vi (x) c + a (x) (b - vi) (x) c */
static void zplus(void) {
  if (R + 1 >= MAXR || R < 2) return;
  const int i = rnd_below(R);
  int j = rnd_below(R - 1);
  if (j >= i) ++j;
  i8 d[32];
  memcpy(d, ZV[j], 32);
  if (!zaxpy(d, -1, ZV[i], KN) || zzero(d, KN)) return;
  memcpy(ZU[R], ZU[j], 32);
  memcpy(ZV[R], d, 32);
  memcpy(ZW[R], ZW[j], 32);
  memcpy(ZV[j], ZV[i], 32);
  znorm(j);
  znorm(R);
  ++R;
}

static int zwalk(int target, long long max_flips, long long plateau, int count) {
  int found = 0;
  long long since = 0;
  zclassical();
  for (int r = 0; r < R; ++r) znorm(r);
  int low = R;
  for (long long f = 0; f < max_flips && found < count; ++f) {
    if ((f & ((1LL << 26) - 1)) == 0 && f) {
      fprintf(stderr, "%lld flips: rank %d, lowest %d\n", f, R, low);
      fflush(stderr);
    }
    if (!zflip()) continue;
    if (zreduce()) since = 0;
    else if (++since > plateau) {
      zplus();
      since = 0;
    }
    if (R < low) low = R;
    if (R <= target) {
      if (!zcheck()) {
        fprintf(stderr, "internal error: scheme fails the Brent equations\n");
        return -1;
      }
      printf("%d", R);
      for (int r = 0; r < R; ++r) {
        putchar(' ');
        for (int x = 0; x < MK; ++x) putchar(ZU[r][x] < 0 ? 'n' : '0' + ZU[r][x]);
        putchar(' ');
        for (int x = 0; x < KN; ++x) putchar(ZV[r][x] < 0 ? 'n' : '0' + ZV[r][x]);
        putchar(' ');
        for (int x = 0; x < MN; ++x) putchar(ZW[r][x] < 0 ? 'n' : '0' + ZW[r][x]);
      }
      putchar('\n');
      fflush(stdout);
      ++found;
      zclassical();
      since = 0;
    }
  }
  return found;
}

int main(int argc, char** argv) {
  if (argc != 9 && argc != 10) {
    fprintf(stderr, "usage: %s M K N target seed max_flips plateau count [z]\n", argv[0]);
    return 2;
  }
  M = atoi(argv[1]);
  K = atoi(argv[2]);
  N = atoi(argv[3]);
  const int target = atoi(argv[4]);
  rng_state = strtoull(argv[5], 0, 10) * 0x9E3779B97F4A7C15ULL + 1;
  const long long max_flips = atoll(argv[6]);
  const long long plateau = atoll(argv[7]);
  const int count = atoi(argv[8]);
  if (M * K > 32 || K * N > 32 || M * N > 32 || M * K * N >= MAXR) {
    fprintf(stderr, "dimensions too large\n");
    return 2;
  }
  if (argc == 10 && argv[9][0] == 'z') {
    MK = M * K;
    KN = K * N;
    MN = M * N;
    const int found = zwalk(target, max_flips, plateau, count);
    fprintf(stderr, "flips done, %d schemes\n", found);
    return found > 0 ? 0 : 1;
  }
  /* Over GF(2) many schemes do not lift to the integers, so once the target
     rank is reached the walk stays there (no plus transitions) and prints a
     scheme every kGap flips: neighbours on the flip graph, each a new
     candidate for lifting. */
  const long long kGap = 1000;
  int found = 0, hit = 0;
  classical();
  long long since = 0, since_print = 0, stuck = 0;
  int best = R;
  for (long long f = 0; f < max_flips && found < count; ++f) {
    if ((f & ((1LL << 26) - 1)) == 0 && f) {
      fprintf(stderr, "%lld flips: rank %d, lowest %d\n", f, R, best);
      fflush(stderr);
    }
    if (!flip()) {
      /* at the target rank with no two terms sharing a factor: no neighbour
         to sample (Strassen's rank-7 schemes are such), so stop */
      if (hit && ++stuck > 1000000) break;
      continue;
    }
    stuck = 0;
    if (reduce()) {
      since = 0;
      if (R < best) best = R;
    } else if (!hit && ++since > plateau) {
      plus();
      since = 0;
    }
    if (R <= target && (!hit || ++since_print >= kGap)) {
      if (!check()) {
        fprintf(stderr, "internal error: scheme fails the tensor check\n");
        return 1;
      }
      printf("%d", R);
      for (int r = 0; r < R; ++r) printf(" %x %x %x", U[r], V[r], W[r]);
      printf("\n");
      fflush(stdout);
      ++found;
      hit = 1;
      since_print = 0;
    }
  }
  fprintf(stderr, "flips done, %d schemes, best rank %d\n", found, best);
  return found ? 0 : 1;
}
