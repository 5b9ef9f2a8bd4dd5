/*
 * zsort_oracle.c -- plain, slow, single-threaded CPU oracle of zSort, the
 * stable distribution sort driven by z-score partitioning
 * ("zSort: Stable Distribution Sort using Z-Score Partitioning",
 * arXiv 2605.14419).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this file.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the GPU implementation.
 *
 * What it computes, step by step in the paper's order (Section III, Proposed
 * Work, and Algorithm 1 "zSort" with its recursive form zsortRec):
 *
 *   1. moments   -- the summation/minimum loop and the variance loop of
 *                   Algorithm 1, kept as exact integers: min o, max M,
 *                   S1 = sum(x - o), S2 = sum((x - o)^2).
 *   2. early exit -- a subproblem whose keys are all identical is solved
 *                   (Section III, duplicate handling; Algorithm 1 "min == mean").
 *   3. statistics -- mean, population standard deviation about the mean in
 *                   use, Zmin = |(min - mean)/std|, scale = clusters/4
 *                   (Algorithm 1), evaluated in IEEE binary64, round to
 *                   nearest even, no contraction, in the fixed order below.
 *   4. map h     -- Eq. (1) with the clip of the cluster definition:
 *                   j = min(floor(((x - mean)/std + Zmin) * scale), k - 1),
 *                   evaluated as fma(x - mean, scale/std, Zmin*scale).
 *   5. histogram, exclusive prefix, stable scatter in input order
 *                   (the three distribution loops of Algorithm 1; one array
 *                   separated by offsets as the text after Algorithm 1 says).
 *   6. per cluster: count <= cutoff -> insertion sort (stable); otherwise
 *                   recurse with the estimated mean
 *                   meanEst = ((j + 0.5)/scale - Zmin) * std + mean
 *                   (Section III, recursive phase zsortRec); k and scale
 *                   are kept for every level (Section III, choice of k).
 *   7. progress guard (a reading, not in the paper): a subproblem uses an
 *                   exact range map (top bits of x - min) once its depth
 *                   reaches max_zlevels, when its parent's z-score pass put
 *                   every key into one cluster, when its statistics are not
 *                   finite, or when its parent used the range map.  The range
 *                   map always splits a non-constant subproblem, so the
 *                   recursion terminates for every input.
 *   8. optional counting sort for a range below a threshold (Section III,
 *                   heuristics paragraph).  Off unless asked for.
 *
 * The final output is the unique stable sort of (key, payload) by unsigned
 * key; steps 1-7 fix every intermediate (statistics bits, histograms, the
 * cluster array after each pass) so that an implementation following the same
 * readings can be compared level by level.
 *
 * Numerics of the statistics (reading of the variance loop, written out):
 *   c   = count, a = RN(S1), nn = RN(c), mu = a / nn
 *   m   = mu at the root; m = meanEst - RN(o_child - o_parent) in a child
 *         (meanEst is computed in the parent's coordinates, where the parent's
 *         minimum is 0; every segment is rebased to its own exact minimum)
 *   D   = c*S2 - S1^2                 (exact integer, >= 0)
 *   var = (RN(D) / nn) / nn + (mu - m) * (mu - m)
 *         -- the identity sum((x-m)^2)/c = D/c^2 + (mu - m)^2, so no
 *            cancellation occurs; at the root mu == m and var = D/c^2.
 *   sigma = sqrt(var); Zmin = |(0 - m) / sigma|; scale = k / 4
 *   A = scale / sigma; B = Zmin * scale
 *
 * Learned partition map (an extension the paper does not have; last section
 * of this file): a monotone MLP 1 -> 32 -> 32 -> 1 fitted to a key sample's
 * CDF -- inference in a fixed precision, cluster ids, thresholds by
 * bisection, the gap-aware piecewise initialisation, the exact binary64
 * squared-error gradient and Adam training.
 *
 * Parity pins for each function are in tests/test_oracle_pins.py and
 * tests/test_oracle_mlp.py; none of the functions here is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------------- */
/* 256-bit unsigned integers, four little-endian 64-bit limbs.             */
/* ---------------------------------------------------------------------- */
typedef struct { uint64_t w[4]; } u256;

static u256 u256_zero(void) { u256 r; memset(&r, 0, sizeof r); return r; }

static u256 u256_from_u128(u128 v)
{
    u256 r = u256_zero();
    r.w[0] = (uint64_t)v;
    r.w[1] = (uint64_t)(v >> 64);
    return r;
}

static u256 u256_add(u256 a, u256 b)
{
    u256 r;
    u128 carry = 0;
    for (int i = 0; i < 4; i++) {
        u128 s = (u128)a.w[i] + b.w[i] + carry;
        r.w[i] = (uint64_t)s;
        carry = s >> 64;
    }
    return r;
}

/* a - b, caller guarantees a >= b */
static u256 u256_sub(u256 a, u256 b)
{
    u256 r;
    uint64_t borrow = 0;
    for (int i = 0; i < 4; i++) {
        u128 t = (u128)a.w[i] - b.w[i] - borrow;
        r.w[i] = (uint64_t)t;
        borrow = (uint64_t)(t >> 64) ? 1 : 0;
    }
    return r;
}

/* a * m, caller guarantees the product fits in 256 bits */
static u256 u256_mul_u64(u256 a, uint64_t m)
{
    u256 r;
    u128 carry = 0;
    for (int i = 0; i < 4; i++) {
        u128 p = (u128)a.w[i] * m + carry;
        r.w[i] = (uint64_t)p;
        carry = p >> 64;
    }
    return r;
}

/* full 128 x 128 -> 256 product, schoolbook on 64-bit limbs */
static u256 u256_mul_u128(u128 a, u128 b)
{
    uint64_t x[2] = { (uint64_t)a, (uint64_t)(a >> 64) };
    uint64_t y[2] = { (uint64_t)b, (uint64_t)(b >> 64) };
    u256 r = u256_zero();
    for (int i = 0; i < 2; i++) {
        u128 carry = 0;
        for (int j = 0; j < 2; j++) {
            u128 p = (u128)x[i] * y[j] + r.w[i + j] + carry;
            r.w[i + j] = (uint64_t)p;
            carry = p >> 64;
        }
        r.w[i + 2] += (uint64_t)carry;
    }
    return r;
}

static int u256_bitlen(u256 a)
{
    for (int i = 3; i >= 0; i--)
        if (a.w[i]) return 64 * i + (64 - __builtin_clzll(a.w[i]));
    return 0;
}

/* bits [s, s+64) of a */
static uint64_t u256_bits64(u256 a, int s)
{
    int q = s / 64, r = s % 64;
    uint64_t lo = q < 4 ? a.w[q] : 0;
    uint64_t hi = q + 1 < 4 ? a.w[q + 1] : 0;
    if (r == 0) return lo;
    return (lo >> r) | (hi << (64 - r));
}

/* any bit below position s set? */
static int u256_any_below(u256 a, int s)
{
    for (int i = 0; i < 4; i++) {
        int lo = 64 * i;
        if (s <= lo) break;
        uint64_t w = a.w[i];
        if (s < lo + 64) w &= (((uint64_t)1) << (s - lo)) - 1;
        if (w) return 1;
    }
    return 0;
}

/*
 * Correctly rounded (nearest, ties to even) conversion of a 256-bit unsigned
 * integer to binary64.  Values below 2^64 use the C conversion, which IEEE 754
 * and C require to round correctly in the default mode.  Larger values keep
 * their top 64 bits with every lower bit folded into bit 0 (a sticky bit):
 * rounding to 53 bits happens at bit 11 of that word, so the fold preserves
 * both the round bit and the "anything below" information, and the final
 * scaling by 2^s is exact.
 */
double zo_u256_to_double(const uint64_t w[4])
{
    u256 a;
    memcpy(a.w, w, sizeof a.w);
    int L = u256_bitlen(a);
    if (L <= 64) return (double)a.w[0];
    int s = L - 64;
    uint64_t top = u256_bits64(a, s);
    if (u256_any_below(a, s)) top |= 1;
    return ldexp((double)top, s);
}

static double u256_to_double(u256 a) { return zo_u256_to_double(a.w); }

/* ---------------------------------------------------------------------- */
/* Step 1: exact moments of a subproblem.                                  */
/* Algorithm 1's first loop (sum, min) and its variance loop, as exact     */
/* integers about the subproblem's own minimum.                            */
/* out: o, M, S1 (2 limbs), S2 (4 limbs)                                   */
/* ---------------------------------------------------------------------- */
void zo_moments(const uint64_t *x, uint64_t n, uint64_t out[8])
{
    uint64_t o = x[0], M = x[0];
    for (uint64_t i = 1; i < n; i++) {
        if (x[i] < o) o = x[i];
        if (x[i] > M) M = x[i];
    }
    u128 s1 = 0;
    u256 s2 = u256_zero();
    for (uint64_t i = 0; i < n; i++) {
        uint64_t d = x[i] - o;
        s1 += d;
        s2 = u256_add(s2, u256_from_u128((u128)d * d));
    }
    out[0] = o;
    out[1] = M;
    out[2] = (uint64_t)s1;
    out[3] = (uint64_t)(s1 >> 64);
    memcpy(out + 4, s2.w, sizeof s2.w);
}

/* ---------------------------------------------------------------------- */
/* Step 3: statistics of the z-score map.                                  */
/* Algorithm 1 (mean, var, std, Zmin, clusters, scale) and Eq. (1).        */
/* is_root: mean from the moments; otherwise m = e - RN(o_rel), where e is */
/* the estimated mean in the parent's coordinates and o_rel = o_child -    */
/* o_parent.                                                               */
/* out: m, var, sigma, zmin, A, B.  Returns 1 if the z-score map is usable */
/* (var > 0 and every parameter finite), 0 otherwise.                      */
/* ---------------------------------------------------------------------- */
int zo_zstats(uint64_t c, const uint64_t s1w[2], const uint64_t s2w[4], int k,
              int is_root, double e, uint64_t o_rel, double out[6])
{
    u128 s1 = ((u128)s1w[1] << 64) | s1w[0];
    u256 s2;
    memcpy(s2.w, s2w, sizeof s2.w);

    /* D = c*S2 - S1^2: c^2 times the population variance about the exact mean */
    u256 cs2 = u256_mul_u64(s2, c);
    u256 s1sq = u256_mul_u128(s1, s1);
    u256 D = u256_sub(cs2, s1sq);

    double nn = (double)c;
    double a = u256_to_double(u256_from_u128(s1));
    double mu = a / nn;
    double m = is_root ? mu : e - (double)o_rel;
    double Dd = u256_to_double(D);
    double v1 = Dd / nn;
    v1 = v1 / nn;
    double dm = mu - m;
    double dm2 = dm * dm;
    double var = v1 + dm2;
    double sigma = sqrt(var);
    double zmin = fabs((0.0 - m) / sigma);
    double scale = (double)k / 4.0;
    double A = scale / sigma;
    double B = zmin * scale;
    out[0] = m; out[1] = var; out[2] = sigma; out[3] = zmin; out[4] = A; out[5] = B;
    if (!(var > 0.0)) return 0;
    if (!isfinite(var) || !isfinite(m) || !isfinite(A) || !isfinite(B)) return 0;
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Step 4: the mapping function h of Eq. (1) with the cluster clip.        */
/* ---------------------------------------------------------------------- */
int zo_zbucket(uint64_t x, uint64_t o, double m, double A, double B, int k)
{
    double xr = (double)(x - o);          /* rebased key, RN */
    double t = fma(xr - m, A, B);         /* ((x - mean)/std + Zmin) * scale */
    double f = floor(t);
    if (!(f >= 0.0)) return 0;            /* rounding below 0, or NaN */
    if (f >= (double)(k - 1)) return k - 1;  /* min(floor(h), k - 1) */
    return (int)f;
}

/* Range map used by the progress guard: the top floor(log2 k) bits of the */
/* key's offset from the minimum, relative to the bit length of the range. */
int zo_rshift(uint64_t R, int k)
{
    int lb = 0;
    while ((2 << lb) <= k) lb++;          /* lb = floor(log2 k) >= 1 */
    int L = R ? 64 - __builtin_clzll(R) : 0;
    return L > lb ? L - lb : 0;
}

int zo_rbucket(uint64_t x, uint64_t o, int shift)
{
    return (int)((x - o) >> shift);
}

/* meanEst of cluster j (recursive phase zsortRec), in the parent's frame */
double zo_mean_est(int j, double scale, double zmin, double sigma, double m)
{
    double q = ((double)j + 0.5) / scale;
    q = q - zmin;
    q = q * sigma;
    return q + m;
}

/* ---------------------------------------------------------------------- */
/* Records of the recursion, one per subproblem larger than the cutoff.    */
/* ---------------------------------------------------------------------- */
typedef struct zo_seg_rec {
    int32_t depth;
    int32_t kind;          /* 1 identical, 2 z-score map, 3 range map, 4 counting sort */
    uint64_t start, count;
    uint64_t o, M;
    uint64_t s1[2];
    uint64_t s2[4];
    double m, sigma, zmin, A, B;
    int32_t shift;
    int32_t nonempty;      /* clusters with at least one key */
    int64_t hist_off;      /* offset of the k counts in the histogram buffer, or -1 */
} zo_seg_rec;

enum { ZO_IDENT = 1, ZO_ZMAP = 2, ZO_RMAP = 3, ZO_COUNT = 4 };

typedef struct zo_params {
    int32_t k;
    int32_t cutoff;
    int32_t max_zlevels;
    int32_t counting_range;   /* 0: off */
} zo_params;

typedef struct ctx {
    uint64_t *keys;
    unsigned char *pay;
    int pw;
    zo_params p;
    zo_seg_rec *tr;
    int64_t tr_cap, tr_n;
    uint32_t *hist;
    int64_t hist_cap, hist_n;
    int64_t max_depth;
    int one_level;            /* stop after the root's pass (level-0 dump) */
} ctx;

static void pay_copy(ctx *c, unsigned char *dst, uint64_t di, const unsigned char *src, uint64_t si)
{
    if (c->pw) memcpy(dst + di * c->pw, src + si * c->pw, (size_t)c->pw);
}

/* stable insertion sort of keys[start, start+n) with payload (Algorithm 1's
 * small-cluster branch) */
static void insertion_sort(ctx *c, uint64_t start, uint64_t n)
{
    uint64_t *x = c->keys + start;
    unsigned char *pay = c->pay ? c->pay + start * c->pw : NULL;
    unsigned char tmp[8];
    for (uint64_t i = 1; i < n; i++) {
        uint64_t key = x[i];
        if (pay) memcpy(tmp, pay + i * c->pw, (size_t)c->pw);
        uint64_t j = i;
        while (j > 0 && x[j - 1] > key) {     /* strict: equal keys keep order */
            x[j] = x[j - 1];
            if (pay) memcpy(pay + j * c->pw, pay + (j - 1) * c->pw, (size_t)c->pw);
            j--;
        }
        x[j] = key;
        if (pay) memcpy(pay + j * c->pw, tmp, (size_t)c->pw);
    }
}

static zo_seg_rec *new_rec(ctx *c, int depth, int kind, uint64_t start, uint64_t n,
                           const uint64_t mom[8])
{
    c->tr_n++;
    if (!c->tr || c->tr_n > c->tr_cap) return NULL;
    zo_seg_rec *r = &c->tr[c->tr_n - 1];
    memset(r, 0, sizeof *r);
    r->depth = depth; r->kind = kind; r->start = start; r->count = n;
    r->o = mom[0]; r->M = mom[1];
    r->s1[0] = mom[2]; r->s1[1] = mom[3];
    memcpy(r->s2, mom + 4, 4 * sizeof(uint64_t));
    r->hist_off = -1;
    return r;
}

/* stable counting sort by x - o (heuristics paragraph of Section III) */
static void counting_sort(ctx *c, uint64_t start, uint64_t n, uint64_t o, uint64_t R)
{
    uint64_t *x = c->keys + start;
    unsigned char *pay = c->pay ? c->pay + start * c->pw : NULL;
    uint64_t bins = R + 1;
    uint64_t *cnt = calloc(bins, sizeof *cnt);
    uint64_t *tk = malloc(n * sizeof *tk);
    unsigned char *tp = pay ? malloc(n * (size_t)c->pw) : NULL;
    for (uint64_t i = 0; i < n; i++) cnt[x[i] - o]++;
    uint64_t run = 0;
    for (uint64_t b = 0; b < bins; b++) { uint64_t t = cnt[b]; cnt[b] = run; run += t; }
    for (uint64_t i = 0; i < n; i++) {
        uint64_t d = cnt[x[i] - o]++;
        tk[d] = x[i];
        if (pay) pay_copy(c, tp, d, pay, i);
    }
    memcpy(x, tk, n * sizeof *tk);
    if (pay) memcpy(pay, tp, n * (size_t)c->pw);
    free(cnt); free(tk); free(tp);
}

static void process(ctx *c, uint64_t start, uint64_t n, int depth, int rmap,
                    double e, uint64_t o_parent, int is_root)
{
    if ((int64_t)depth > c->max_depth) c->max_depth = depth;
    if (n <= (uint64_t)c->p.cutoff) {
        insertion_sort(c, start, n);
        return;
    }
    uint64_t *x = c->keys + start;
    unsigned char *pay = c->pay ? c->pay + start * c->pw : NULL;
    const int k = c->p.k;

    /* step 1 */
    uint64_t mom[8];
    zo_moments(x, n, mom);
    uint64_t o = mom[0], M = mom[1];

    /* step 2: all keys identical -> already sorted, input order kept */
    if (o == M) {
        new_rec(c, depth, ZO_IDENT, start, n, mom);
        return;
    }
    /* step 8 (optional) */
    if (c->p.counting_range > 0 && M - o < (uint64_t)c->p.counting_range) {
        new_rec(c, depth, ZO_COUNT, start, n, mom);
        counting_sort(c, start, n, o, M - o);
        return;
    }

    /* step 3 */
    double st[6] = {0, 0, 0, 0, 0, 0};
    if (!rmap) {
        int ok = zo_zstats(n, mom + 2, mom + 4, k, is_root, e, o - o_parent, st);
        if (!ok) rmap = 1;
    }
    int shift = rmap ? zo_rshift(M - o, k) : 0;
    double m = st[0], sigma = st[2], zmin = st[3], A = st[4], B = st[5];
    double scale = (double)k / 4.0;

    /* step 5: histogram (third loop of Algorithm 1) */
    uint64_t *cnt = calloc((size_t)k, sizeof *cnt);
    for (uint64_t i = 0; i < n; i++) {
        int b = rmap ? zo_rbucket(x[i], o, shift) : zo_zbucket(x[i], o, m, A, B, k);
        cnt[b]++;
    }
    /* exclusive prefix */
    uint64_t *off = malloc((size_t)k * sizeof *off);
    uint64_t run = 0;
    for (int b = 0; b < k; b++) { off[b] = run; run += cnt[b]; }
    /* stable scatter in input order into the cluster array, then back into
     * the subproblem's range (one array separated by offsets) */
    uint64_t *tk = malloc(n * sizeof *tk);
    unsigned char *tp = pay ? malloc(n * (size_t)c->pw) : NULL;
    uint64_t *pos = malloc((size_t)k * sizeof *pos);
    memcpy(pos, off, (size_t)k * sizeof *pos);
    for (uint64_t i = 0; i < n; i++) {
        int b = rmap ? zo_rbucket(x[i], o, shift) : zo_zbucket(x[i], o, m, A, B, k);
        uint64_t d = pos[b]++;
        tk[d] = x[i];
        if (pay) pay_copy(c, tp, d, pay, i);
    }
    memcpy(x, tk, n * sizeof *tk);
    if (pay) memcpy(pay, tp, n * (size_t)c->pw);
    free(tk); free(tp); free(pos);

    zo_seg_rec *r = new_rec(c, depth, rmap ? ZO_RMAP : ZO_ZMAP, start, n, mom);
    if (r) {
        r->m = m; r->sigma = sigma; r->zmin = zmin; r->A = A; r->B = B; r->shift = shift;
        int ne = 0;
        for (int b = 0; b < k; b++) ne += cnt[b] > 0;
        r->nonempty = ne;
        if (c->hist && c->hist_n + k <= c->hist_cap) {
            r->hist_off = c->hist_n;
            for (int b = 0; b < k; b++) c->hist[c->hist_n + b] = (uint32_t)cnt[b];
            c->hist_n += k;
        }
    }

    /* step 6: every non-empty cluster in order */
    if (!c->one_level) {
        for (int j = 0; j < k; j++) {
            if (!cnt[j]) continue;
            int child_rmap = rmap || depth + 1 >= c->p.max_zlevels || cnt[j] == n;
            double ce = child_rmap ? 0.0 : zo_mean_est(j, scale, zmin, sigma, m);
            process(c, start + off[j], cnt[j], depth + 1, child_rmap, ce, o, 0);
        }
    }
    free(cnt); free(off);
}

static int check_params(const zo_params *p)
{
    if (p->k < 2 || p->k > (1 << 20)) return -1;
    if (p->cutoff < 1) return -1;
    if (p->max_zlevels < 0) return -1;
    if (p->counting_range < 0) return -1;
    return 0;
}

/*
 * Sort keys[0, n) (unsigned, ascending, stable) carrying pw-byte payloads
 * (pw in {0, 4, 8}; payload may be NULL when pw == 0).  Records of the
 * subproblems larger than the cutoff are written to tr (up to tr_cap) and
 * their histograms to hist (up to hist_cap counts).  info[0] = records
 * produced (may exceed tr_cap), info[1] = histogram counts stored,
 * info[2] = deepest level reached.  Returns 0, or -1 for bad arguments.
 */
int zo_sort(uint64_t *keys, void *payload, int pw, uint64_t n, const zo_params *p,
            zo_seg_rec *tr, int64_t tr_cap, uint32_t *hist, int64_t hist_cap,
            int64_t info[3])
{
    if (check_params(p) || (pw != 0 && pw != 4 && pw != 8) || (pw && !payload)) return -1;
    ctx c;
    memset(&c, 0, sizeof c);
    c.keys = keys; c.pay = payload; c.pw = pw; c.p = *p;
    c.tr = tr; c.tr_cap = tr_cap; c.hist = hist; c.hist_cap = hist_cap;
    if (n > 1) process(&c, 0, n, 0, p->max_zlevels == 0, 0.0, 0, 1);
    if (info) { info[0] = c.tr_n; info[1] = c.hist_n; info[2] = c.max_depth; }
    return 0;
}

/* One distribution pass over the whole array (the root), no recursion:
 * keys/payload become Algorithm 1's cluster array.  The root record and its
 * histogram are returned as in zo_sort.  Requires n > cutoff. */
int zo_level0(uint64_t *keys, void *payload, int pw, uint64_t n, const zo_params *p,
              zo_seg_rec *tr, uint32_t *hist, int64_t hist_cap)
{
    if (check_params(p) || (pw != 0 && pw != 4 && pw != 8) || (pw && !payload)) return -1;
    if (n <= (uint64_t)p->cutoff) return -1;
    ctx c;
    memset(&c, 0, sizeof c);
    c.keys = keys; c.pay = payload; c.pw = pw; c.p = *p;
    c.tr = tr; c.tr_cap = 1; c.hist = hist; c.hist_cap = hist_cap;
    c.one_level = 1;
    process(&c, 0, n, 0, p->max_zlevels == 0, 0.0, 0, 1);
    return 0;
}

/* Independent segments: each [off[i], off[i+1]) is sorted on its own. */
int zo_sort_segmented(uint64_t *keys, void *payload, int pw, uint64_t n,
                      const int64_t *off, int64_t nseg, const zo_params *p)
{
    if (check_params(p) || (pw != 0 && pw != 4 && pw != 8) || (pw && !payload)) return -1;
    if (nseg < 0 || (nseg > 0 && (off[0] != 0 || (uint64_t)off[nseg] != n))) return -1;
    for (int64_t i = 0; i < nseg; i++)
        if (off[i + 1] < off[i]) return -1;
    unsigned char *pay = payload;
    for (int64_t i = 0; i < nseg; i++) {
        uint64_t s = (uint64_t)off[i], len = (uint64_t)(off[i + 1] - off[i]);
        int rc = zo_sort(keys + s, pay ? pay + s * pw : NULL, pw, len, p, NULL, 0, NULL, 0, NULL);
        if (rc) return rc;
    }
    return 0;
}

/*
 * Brute force, independent of everything above: output position by position,
 * take the smallest remaining key, the earliest one among equals.  O(n^2).
 */
int zo_brute_stable_sort(uint64_t *keys, void *payload, int pw, uint64_t n)
{
    if ((pw != 0 && pw != 4 && pw != 8) || (pw && !payload)) return -1;
    unsigned char *pay = payload;
    unsigned char *used = calloc(n ? n : 1, 1);
    uint64_t *ok = malloc((n ? n : 1) * sizeof *ok);
    unsigned char *op = pw ? malloc((n ? n : 1) * (size_t)pw) : NULL;
    for (uint64_t pos = 0; pos < n; pos++) {
        uint64_t best = n;
        for (uint64_t i = 0; i < n; i++) {
            if (used[i]) continue;
            if (best == n || keys[i] < keys[best]) best = i;
        }
        used[best] = 1;
        ok[pos] = keys[best];
        if (pw) memcpy(op + pos * pw, pay + best * pw, (size_t)pw);
    }
    memcpy(keys, ok, n * sizeof *ok);
    if (pw) memcpy(pay, op, n * (size_t)pw);
    free(used); free(ok); free(op);
    return 0;
}

int zo_seg_rec_size(void) { return (int)sizeof(zo_seg_rec); }

/* ====================================================================== */
/* 128-bit keys (an extension: the paper motivates key widths beyond 64   */
/* bits, Section I).  The result has a plain definition, written out here: */
/* the stable sort of the (key, payload) pairs by the unsigned 128-bit key  */
/* (hi, lo), or by the signed one (hi compared with its sign bit flipped).  */
/* keys holds 2n words, low word first per key.  A bottom-up merge sort   */
/* that takes from the left run on ties is stable.                        */
/* ====================================================================== */
static int key128_less(const uint64_t *a, const uint64_t *b, int sgn)
{
    uint64_t ah = a[1] ^ (sgn ? 0x8000000000000000ull : 0), bh = b[1] ^ (sgn ? 0x8000000000000000ull : 0);
    if (ah != bh) return ah < bh;
    return a[0] < b[0];
}

int zo_sort128(uint64_t *keys, uint32_t *payload, uint64_t n, int sgn)
{
    if (n < 2) return 0;
    uint64_t *tk = malloc(n * 2 * sizeof *tk);
    uint32_t *tp = payload ? malloc(n * sizeof *tp) : NULL;
    if (!tk || (payload && !tp)) { free(tk); free(tp); return -1; }
    uint64_t *src = keys, *dst = tk;
    uint32_t *ps = payload, *pd = tp;
    for (uint64_t w = 1; w < n; w *= 2) {
        for (uint64_t lo = 0; lo < n; lo += 2 * w) {
            uint64_t mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
            uint64_t i = lo, j = mid, o = lo;
            while (i < mid || j < hi) {
                int take_right = j < hi && (i >= mid || key128_less(src + 2 * j, src + 2 * i, sgn));
                uint64_t f = take_right ? j++ : i++;
                dst[2 * o] = src[2 * f];
                dst[2 * o + 1] = src[2 * f + 1];
                if (payload) pd[o] = ps[f];
                o++;
            }
        }
        uint64_t *t = src; src = dst; dst = t;
        uint32_t *u = ps; ps = pd; pd = u;
    }
    if (src != keys) {
        memcpy(keys, src, n * 2 * sizeof *keys);
        if (payload) memcpy(payload, ps, n * sizeof *payload);
    }
    free(tk);
    free(tp);
    return 0;
}

/* ====================================================================== */
/* Learned partition (an extension beyond the paper): a monotone MLP that  */
/* approximates the keys' CDF and replaces the z-score map at the first    */
/* pass.  Parameters, 1153 values in this order: W1[32] b1[32] W2[32][32]  */
/* (row = output unit) b2[32] W3[32] b3.  W1 and b1 are binary64 (a ramp   */
/* of the first layer must be placed to within a fraction of its width, and */
/* a narrow, heavy mixture component far from 0 spans ~1e-7 of the        */
/* normalised range, below binary32's resolution); the rest are binary32  */
/* values, passed here as doubles that binary32 represents exactly.        */
/* Non-negative weights and clamp ramps make f non-decreasing.             */
/* ====================================================================== */
enum { ZO_H = 32, ZO_NP = 1153, ZO_W1 = 0, ZO_B1 = 32, ZO_W2 = 64, ZO_B2 = 1088, ZO_W3 = 1120,
       ZO_B3 = 1152 };

static float clamp01f(float a) { return a < 0.0f ? 0.0f : (a > 1.0f ? 1.0f : a); }

/* normalised key: 0 at or below smin, 1 at or above smax, else the ratio */
double zo_mlp_norm(uint64_t x, uint64_t smin, uint64_t smax)
{
    if (x <= smin) return 0.0;
    if (x >= smax) return 1.0;
    return (double)(x - smin) / (double)(smax - smin);
}

/* Inference in the precision both sides use: the first layer in binary64
 * (product, then sum), rounded once to binary32; everything after in
 * binary32, products and sums rounded separately, sums in index order. */
float zo_mlp_forward(const double *p, double u)
{
    float h1[ZO_H], h2[ZO_H];
    for (int i = 0; i < ZO_H; i++) {
        double a = p[ZO_W1 + i] * u;
        a = a + p[ZO_B1 + i];
        h1[i] = clamp01f((float)a);
    }
    for (int j = 0; j < ZO_H; j++) {
        float acc = (float)p[ZO_B2 + j];
        for (int i = 0; i < ZO_H; i++) {
            float t = (float)p[ZO_W2 + j * ZO_H + i] * h1[i];
            acc = acc + t;
        }
        h2[j] = clamp01f(acc);
    }
    float f = (float)p[ZO_B3];
    for (int j = 0; j < ZO_H; j++) {
        float t = (float)p[ZO_W3 + j] * h2[j];
        f = f + t;
    }
    return f;
}

/* cluster of a key under the learned map with B clusters */
int zo_mlp_bucket(const double *p, uint64_t x, uint64_t smin, uint64_t smax, int B)
{
    float f = clamp01f(zo_mlp_forward(p, zo_mlp_norm(x, smin, smax)));
    float t = (float)B * f;
    float fl = floorf(t);
    if (fl >= (float)(B - 1)) return B - 1;
    return (int)fl;
}

/* Thresholds t_b = min{x : bucket(x) >= b} for b = 1..nt, where
 * nt = bucket(2^64 - 1); found by bisection over the u64 keys, which is
 * exact when the map is non-decreasing.  Returns nt; out gets B-1 words
 * (unused ones are 0). */
int zo_mlp_thresholds(const double *p, uint64_t smin, uint64_t smax, int B, uint64_t *out)
{
    int nt = zo_mlp_bucket(p, UINT64_MAX, smin, smax, B);
    for (int b = 1; b < B; b++) out[b - 1] = 0;
    for (int b = 1; b <= nt; b++) {
        uint64_t lo = 0, hi = UINT64_MAX;   /* bucket(hi) >= b */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (zo_mlp_bucket(p, mid, smin, smax, B) >= b) hi = mid;
            else lo = mid + 1;
        }
        out[b - 1] = lo;
    }
    return nt;
}

/* Initialisation from the sorted sample s[0, m) (u = normalised keys).
 * The sample is cut into ZO_NBLK blocks of equal count; a block whose
 * largest gap between consecutive keys covers more than half of its key
 * range is cut at that gap (at most ZO_NSPLIT blocks, those with the largest
 * gap-to-range ratio, ties to the lower block).  Each piece r of consecutive
 * sample keys [a, b] gets one unit of the first layer, a ramp from 0 at u[a]
 * to 1 at u[b] (a step at u[a] when u[a] == u[b]); the second layer passes
 * the ramps through and the output weighs ramp r by its share (b - a + 1)/m
 * of the sample.  f is then the sample CDF interpolated linearly inside each
 * piece and flat between pieces, so a gap between two mixture components
 * gets no clusters.  Unused units stay 0. */
enum { ZO_NBLK = 28, ZO_NSPLIT = 4 };

void zo_mlp_init(const uint64_t *s, uint64_t m, uint64_t smin, uint64_t smax, double *p)
{
    for (int i = 0; i < ZO_NP; i++) p[i] = 0.0;
    uint64_t lo[ZO_NBLK + 1];
    for (int i = 0; i <= ZO_NBLK; i++) lo[i] = ((uint64_t)i * m) / ZO_NBLK;
    double score[ZO_NBLK];
    uint64_t cut[ZO_NBLK];
    for (int i = 0; i < ZO_NBLK; i++) {
        score[i] = 0.0;
        cut[i] = 0;
        uint64_t a = lo[i], b = lo[i + 1];
        if (b - a < 2) continue;
        double span = zo_mlp_norm(s[b - 1], smin, smax) - zo_mlp_norm(s[a], smin, smax);
        if (!(span > 0.0)) continue;
        double gmax = -1.0;
        for (uint64_t j = a; j + 1 < b; j++) {
            double g = zo_mlp_norm(s[j + 1], smin, smax) - zo_mlp_norm(s[j], smin, smax);
            if (g > gmax) { gmax = g; cut[i] = j; }
        }
        score[i] = gmax / span;
    }
    int split[ZO_NBLK];
    for (int i = 0; i < ZO_NBLK; i++) split[i] = 0;
    for (int k = 0; k < ZO_NSPLIT; k++) {
        int best = -1;
        for (int i = 0; i < ZO_NBLK; i++)
            if (!split[i] && score[i] > 0.5 && (best < 0 || score[i] > score[best])) best = i;
        if (best < 0) break;
        split[best] = 1;
    }
    int r = 0;
    for (int i = 0; i < ZO_NBLK; i++) {
        uint64_t a = lo[i], b = lo[i + 1];
        if (a == b) continue;
        uint64_t piece[2][2];
        int np_ = 0;
        if (split[i]) {
            piece[0][0] = a; piece[0][1] = cut[i];
            piece[1][0] = cut[i] + 1; piece[1][1] = b - 1;
            np_ = 2;
        } else {
            piece[0][0] = a; piece[0][1] = b - 1;
            np_ = 1;
        }
        for (int q = 0; q < np_; q++, r++) {
            double ua = zo_mlp_norm(s[piece[q][0]], smin, smax);
            double ub = zo_mlp_norm(s[piece[q][1]], smin, smax);
            double w = ub > ua ? 1.0 / (ub - ua) : 4503599627370496.0;  /* 2^52: a step */
            p[ZO_W1 + r] = w;
            p[ZO_B1 + r] = -ua * w;
            p[ZO_W2 + r * ZO_H + r] = 1.0;
            p[ZO_W3 + r] = (double)(float)((double)(piece[q][1] - piece[q][0] + 1) / (double)m);
        }
    }
}

/* Mean squared error over (u[s], y[s]) and its exact gradient in binary64
 * (the clamp's derivative is 1 strictly inside (0, 1), else 0); binary32
 * parameters enter as the doubles they are. */
double zo_mlp_loss_grad(const double *p, const double *u, const double *y, uint64_t m, double *g)
{
    double W1[ZO_H], b1[ZO_H], W2[ZO_H][ZO_H], b2[ZO_H], W3[ZO_H], b3 = p[ZO_B3];
    for (int i = 0; i < ZO_H; i++) {
        W1[i] = p[ZO_W1 + i]; b1[i] = p[ZO_B1 + i]; b2[i] = p[ZO_B2 + i]; W3[i] = p[ZO_W3 + i];
        for (int k = 0; k < ZO_H; k++) W2[i][k] = p[ZO_W2 + i * ZO_H + k];
    }
    if (g) for (int i = 0; i < ZO_NP; i++) g[i] = 0.0;
    double loss = 0.0;
    for (uint64_t s = 0; s < m; s++) {
        double a1[ZO_H], h1[ZO_H], a2[ZO_H], h2[ZO_H];
        for (int i = 0; i < ZO_H; i++) {
            a1[i] = W1[i] * u[s] + b1[i];
            h1[i] = a1[i] < 0 ? 0 : (a1[i] > 1 ? 1 : a1[i]);
        }
        for (int j = 0; j < ZO_H; j++) {
            a2[j] = b2[j];
            for (int i = 0; i < ZO_H; i++) a2[j] += W2[j][i] * h1[i];
            h2[j] = a2[j] < 0 ? 0 : (a2[j] > 1 ? 1 : a2[j]);
        }
        double f = b3;
        for (int j = 0; j < ZO_H; j++) f += W3[j] * h2[j];
        double r = f - y[s];
        loss += r * r / (double)m;
        if (!g) continue;
        double e = 2.0 * r / (double)m;
        double d2[ZO_H], d1[ZO_H];
        g[ZO_B3] += e;
        for (int j = 0; j < ZO_H; j++) {
            g[ZO_W3 + j] += e * h2[j];
            d2[j] = (a2[j] > 0 && a2[j] < 1) ? e * W3[j] : 0.0;
            g[ZO_B2 + j] += d2[j];
        }
        for (int i = 0; i < ZO_H; i++) {
            double acc = 0.0;
            for (int j = 0; j < ZO_H; j++) {
                g[ZO_W2 + j * ZO_H + i] += d2[j] * h1[i];
                acc += d2[j] * W2[j][i];
            }
            d1[i] = (a1[i] > 0 && a1[i] < 1) ? acc : 0.0;
            g[ZO_B1 + i] += d1[i];
            g[ZO_W1 + i] += d1[i] * u[s];
        }
    }
    return loss;
}

/* Training of the map: Adam (Kingma and Ba, "Adam: A Method for Stochastic
 * Optimization", ICLR 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and
 * bias correction, on the mean squared error of minibatch j = t mod nb
 * (samples j, j + nb, j + 2nb, ...) at step t; exact binary64 gradients;
 * W1 and b1 stay binary64, every other parameter is rounded to binary32
 * after each step; weights (not biases) are projected onto >= 0.
 * Returns the loss of the last step's minibatch (before its update);
 * *loss_first gets the first step's. */
double zo_mlp_train(double *p, const double *u, const double *y, uint64_t m, uint32_t nb,
                    uint32_t steps, double lr, double *loss_first)
{
    double m1[ZO_NP], m2[ZO_NP], g[ZO_NP];
    for (int i = 0; i < ZO_NP; i++) m1[i] = m2[i] = 0.0;
    double *ub = (double *)malloc(sizeof(double) * (m / nb + 1));
    double *yb = (double *)malloc(sizeof(double) * (m / nb + 1));
    double b1p = 1.0, b2p = 1.0, last = 0.0;
    for (uint32_t t = 0; t < steps; t++) {
        uint32_t j = t % nb;
        uint64_t c = 0;
        for (uint64_t i = j; i < m; i += nb) { ub[c] = u[i]; yb[c] = y[i]; c++; }
        double loss = c ? zo_mlp_loss_grad(p, ub, yb, c, g) : 0.0;
        if (t == 0 && loss_first) *loss_first = loss;
        last = loss;
        b1p = b1p * 0.9;
        b2p = b2p * 0.999;
        for (int i = 0; i < ZO_NP; i++) {
            m1[i] = 0.9 * m1[i] + (1.0 - 0.9) * g[i];
            m2[i] = 0.999 * m2[i] + (1.0 - 0.999) * (g[i] * g[i]);
            double mh = m1[i] / (1.0 - b1p);
            double vh = m2[i] / (1.0 - b2p);
            double pn = p[i] - (lr * mh) / (sqrt(vh) + 1e-8);
            int weight = (i < ZO_B1) || (i >= ZO_W2 && i < ZO_B2) || (i >= ZO_W3 && i < ZO_B3);
            if (weight && !(pn > 0.0)) pn = 0.0;
            p[i] = i < ZO_W2 ? pn : (double)(float)pn;
        }
    }
    free(ub);
    free(yb);
    return last;
}
