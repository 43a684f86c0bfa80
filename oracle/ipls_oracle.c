/*
 * IPLS oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU implementation of what the In-Place Parallel Learned Sort
 * (IPLS) distribution recursion computes.  It exists so that tests, the smoke check and the
 * bench's CPU-baseline leg have something independent to compare the GPU library against.
 * Nothing in the product path may link, load or call it, and it shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math (no FMA contraction:
 * every fp64 operation below is rounded exactly where it is written).
 *
 * What it computes, with the passage each step follows:
 *   - key map (Experimental Evaluation: doubles are sorted through an order-preserving map to
 *     unsigned integers); keys are ordered by IEEE 754 totalOrder;
 *   - sample of a bucket (Background, IPS4o section: partitioning starts by sampling; Learned
 *     Sort section: a 1% sample works well);
 *   - sort of the sample (Machine Learning Models chapter: the sample is sorted by another
 *     algorithm; the sorted sample is unique, so any sort gives the same bits);
 *   - FMCD fit (Linear Models section: the smallest conflict degree D), in fp64;
 *   - the clamped linear partition model (Linear Models section, the piecewise F(x));
 *   - stable distribution into contiguous buckets (Proposed Algorithm, Worked Example: the
 *     layout after "a pass to make the buckets contiguous" is the stable counting-sort layout);
 *   - recursion on buckets above the base-case size, base case below it (Proposed Algorithm);
 *   - homogeneous buckets are left as they are (Learned Sort section, Learned Sort 2.0's
 *     homogeneity check); a degenerate fit falls back to a most-significant-digit split
 *     (IPS4o section, IPS2Ra's radix partitioning);
 *   - the two-level piecewise-linear CDF model (Recursive Model Index section, eCDF models
 *     trained by mean-squared error in the Machine Learning Models chapter).  Parity unpinned
 *     for this model beyond its definition: the paper prints no numbers for it;
 *   - equality buckets and the splitter tree (IPS4o's, Decision Trees section);
 *   - sample inheritance (an extension inside the Machine Learning Models chapter's
 *     sample -> sort -> train -> predict pipeline, not described by the paper): a child bucket
 *     may reuse its part of the parent's sorted sample instead of drawing a fresh one.  Pinned
 *     by the rule written out in numpy (restricted samples, sizes, usable fits) and by sorts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_F64 0
#define OR_F32 1
#define OR_U64 2

#define MODEL_LINEAR 0
#define MODEL_MSD 1
#define MODEL_CLOSED 2
#define MODEL_L2PL 3
#define MODEL_TREE 4

typedef struct {
    uint32_t num_buckets;    /* K */
    uint32_t base_case_max;  /* T: a bucket of n <= T keys goes to the base case */
    uint32_t sample_divisor; /* S = ceil(n / divisor) ... */
    uint32_t sample_min;     /* ... but at least this (0 means 2K) ... */
    uint64_t sample_max;     /* ... and at most this (0 means no cap), never above n */
    uint64_t seed;           /* jitter of the sample positions */
    uint32_t model;          /* 0 FMCD, 1 auto (two-level model iff lower max sample load), 2 two-level,
                              * 3 splitter tree */
    uint32_t leaves;         /* M leaves of the two-level model */
    uint32_t train_iters;    /* gradient steps of the two-level model */
    uint32_t sample_policy;  /* 0: S = ceil(n / divisor); 1: the paper's alpha*K - 1 */
    uint32_t equality;       /* 1: equality buckets for heavy sample values (IPS4o) */
    uint32_t inherit;        /* 1: a child bucket reuses its part of the parent's sorted sample */
    uint32_t bucket_policy;  /* 1: fewer buckets for small buckets (bucket_count) */
} oracle_params;

typedef struct {
    uint32_t kind; /* MODEL_* */
    uint32_t K;
    double a, b;   /* linear model: t = fma(a, val, b) */
    uint64_t D;    /* FMCD's conflict degree */
    uint64_t umin; /* MSD fallback: c = (ord - umin) >> shift */
    uint32_t shift;
    uint32_t degenerate;
    uint64_t S; /* sample size the model was fitted on */
    uint64_t max_load_linear; /* max sample load of the FMCD model (model=auto only) */
    uint64_t max_load_l2pl;   /* max sample load of the two-level model (model=auto only) */
    uint32_t neq;             /* equality buckets: number of heavy sample values (0 = none) */
    uint32_t Km;              /* buckets of the linear part when neq > 0: K - 2 neq */
    uint32_t const0;          /* linear part unusable: every other key is in linear bucket 0 */
    uint32_t pad_;
    uint64_t heavy[16];       /* the heavy values' ords, ascending */
    uint32_t tree_strict;     /* splitter tree: bucket = #{splitters < key} (1) or <= key (0) */
    uint32_t pad2_;
    uint64_t split[255];      /* splitter tree: the K-1 splitters' ords, ascending */
} oracle_model;

typedef struct {
    uint64_t passes;     /* buckets partitioned */
    uint64_t max_level;  /* deepest level that was partitioned, 1 = the whole array */
    uint64_t closed;     /* buckets closed by the homogeneity check */
    uint64_t fallback;   /* buckets split by the MSD digit */
    uint64_t base_cases; /* base-case sorts of more than one key */
    uint64_t l2pl_used;  /* partitions that used the two-level model */
    uint64_t level1_max_load;
    uint64_t keys_partitioned; /* sum of the sizes of the partitioned buckets */
    uint64_t inherited;        /* partitioned buckets whose model came from the parent's sample */
} oracle_stats;

/* ---------------------------------------------------------------- key map */

static size_t key_bytes(int dtype) { return dtype == OR_F32 ? 4 : 8; }

/* IEEE 754 totalOrder as an unsigned integer: flip every bit of a negative number, set the
 * sign bit of a positive one.  -0 < +0, -NaN below -inf, +NaN above +inf. */
uint64_t oracle_ord_one(const void* keys, size_t i, int dtype) {
    if (dtype == OR_F32) {
        uint32_t u;
        memcpy(&u, (const char*)keys + 4 * i, 4);
        return (u & 0x80000000u) ? (uint64_t)(uint32_t)~u : (uint64_t)(u | 0x80000000u);
    }
    uint64_t u;
    memcpy(&u, (const char*)keys + 8 * i, 8);
    if (dtype == OR_U64) return u;
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

/* The value the model sees: fp64 as is, fp32 widened (exact), u64 rounded to nearest even. */
double oracle_val_one(const void* keys, size_t i, int dtype) {
    if (dtype == OR_F32) {
        float f;
        memcpy(&f, (const char*)keys + 4 * i, 4);
        return (double)f;
    }
    if (dtype == OR_U64) {
        uint64_t u;
        memcpy(&u, (const char*)keys + 8 * i, 8);
        return (double)u;
    }
    double d;
    memcpy(&d, (const char*)keys + 8 * i, 8);
    return d;
}

static int key_negative(const void* keys, size_t i, int dtype) {
    if (dtype == OR_U64) return 0;
    if (dtype == OR_F32) {
        uint32_t u;
        memcpy(&u, (const char*)keys + 4 * i, 4);
        return (int)(u >> 31);
    }
    uint64_t u;
    memcpy(&u, (const char*)keys + 8 * i, 8);
    return (int)(u >> 63);
}

void oracle_keymap(const void* keys, size_t n, int dtype, uint64_t* ord_out, double* val_out) {
    for (size_t i = 0; i < n; ++i) {
        if (ord_out) ord_out[i] = oracle_ord_one(keys, i, dtype);
        if (val_out) val_out[i] = oracle_val_one(keys, i, dtype);
    }
}

/* ---------------------------------------------------------------- sample */

/* SplitMix64's output function (Steele, Lea, Flood 2014), used as a counter-based hash. */
uint64_t oracle_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

#define GOLDEN_GAMMA 0x9e3779b97f4a7c15ull

/* Sample size of a bucket of n keys: ceil(n / divisor), raised to sample_min (2K by default),
 * capped by sample_max when given, and never more than n.  The paper's Learned Sort section
 * reports a 1% sample (divisor 100) as a good choice. */
/* Binary logarithm of n >= 1: the exponent, plus 24 fractional bits obtained by squaring the
 * mantissa m in [1, 2) repeatedly (each squaring that reaches 2 contributes the next bit). */
double oracle_log2(uint64_t n) {
    int e = 63 - __builtin_clzll(n);
    double m = ldexp((double)n, -e);
    if (m >= 2.0) { /* (double)n rounded up to the next power of two */
        m = m / 2.0;
        e = e + 1;
    }
    double f = 0.0, bit = 0.5;
    for (int i = 0; i < 24; ++i) {
        m = m * m;
        if (m >= 2.0) {
            m = m / 2.0;
            f = f + bit;
        }
        bit = bit / 2.0;
    }
    return (double)e + f;
}

/* Sample size of a bucket of n keys.
 * Policy 0 (Learned Sort's 1%, Background chapter): ceil(n / divisor), at least sample_min
 *   (0 means 2K).
 * Policy 1 (IPLS, Proposed Algorithm chapter): alpha*K - 1 with alpha = 0.2 log2(n), rounded
 *   to the nearest integer (halves down), at least sample_min when that is non-zero, and at
 *   most ceil(n/2) so that a sample is always smaller than its bucket.
 * Both: at most sample_max when non-zero, never above n. */
uint64_t oracle_sample_size(uint64_t n, const oracle_params* p) {
    uint64_t s;
    if (p->sample_policy == 1) {
        double t = 0.2 * oracle_log2(n ? n : 1) * (double)p->num_buckets - 0.5;
        s = t > 0.0 ? (uint64_t)t : 0;
        if (p->sample_min && s < p->sample_min) s = p->sample_min;
        if (s > (n + 1) / 2) s = (n + 1) / 2;
    } else {
        uint64_t div = p->sample_divisor ? p->sample_divisor : 100;
        uint64_t smin = p->sample_min ? p->sample_min : 2ull * p->num_buckets;
        s = (n + div - 1) / div;
        if (s < smin) s = smin;
    }
    if (p->sample_max && s > p->sample_max) s = p->sample_max;
    if (s > n) s = n;
    return s;
}

/* One position per stratum j = [floor(j n / S), floor((j+1) n / S)), moved inside the stratum
 * by a hash of (seed, bucket offset within its array, bucket size, j).  Positions are relative
 * to the bucket start. */
void oracle_sample_positions(uint64_t n, uint64_t lo_rel, uint64_t S, uint64_t seed, uint64_t* pos) {
    uint64_t stream = oracle_mix64(seed ^ oracle_mix64(lo_rel * GOLDEN_GAMMA + n));
    for (uint64_t j = 0; j < S; ++j) {
        uint64_t a = (uint64_t)(((unsigned __int128)j * n) / S);
        uint64_t b = (uint64_t)(((unsigned __int128)(j + 1) * n) / S);
        uint64_t h = oracle_mix64(stream + (j + 1) * GOLDEN_GAMMA);
        pos[j] = a + h % (b - a);
    }
}

static int cmp_u64(const void* pa, const void* pb) {
    uint64_t a = *(const uint64_t*)pa, b = *(const uint64_t*)pb;
    return (a > b) - (a < b);
}

/* Value of an ord-mapped key (inverse key map followed by val). */
static double val_from_ord(uint64_t o, int dtype) {
    if (dtype == OR_U64) return (double)o;
    if (dtype == OR_F32) {
        uint32_t u = (uint32_t)o;
        u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
        float f;
        memcpy(&f, &u, 4);
        return (double)f;
    }
    uint64_t u = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    double d;
    memcpy(&d, &u, 8);
    return d;
}

/* Sorted sample of a bucket as fp64 values x[0..S): gather, sort by ord, map to val. */
/* The sorted sample as ords (ords_out, nullable) and as the fp64 values the models see (x). */
static void sorted_sample_ords(const void* keys, uint64_t n, int dtype, uint64_t lo_rel, uint64_t S, uint64_t seed,
                               double* x, uint64_t* ords_out) {
    uint64_t* pos = (uint64_t*)malloc((S ? S : 1) * sizeof(uint64_t));
    uint64_t* ords = (uint64_t*)malloc((S ? S : 1) * sizeof(uint64_t));
    oracle_sample_positions(n, lo_rel, S, seed, pos);
    for (uint64_t j = 0; j < S; ++j) ords[j] = oracle_ord_one(keys, pos[j], dtype);
    qsort(ords, S, sizeof(uint64_t), cmp_u64);
    for (uint64_t j = 0; j < S; ++j) x[j] = val_from_ord(ords[j], dtype);
    if (ords_out) memcpy(ords_out, ords, S * sizeof(uint64_t));
    free(pos);
    free(ords);
}

void oracle_sorted_sample(const void* keys, uint64_t n, int dtype, uint64_t lo_rel, uint64_t S, uint64_t seed,
                          double* x) {
    sorted_sample_ords(keys, n, dtype, lo_rel, S, seed, x, NULL);
}

/* ---------------------------------------------------------------- FMCD (Linear Models section) */

/* u(D): the spread that every window of D+1 consecutive sample keys must reach, namely the
 * range of the sample with D keys cut from each end, over K-2 gaps. */
static double fmcd_spread(const double* x, uint64_t S, uint64_t D, uint32_t K) {
    return (x[S - 1 - D] - x[D]) / (double)(K - 2);
}

/* The conflict-degree condition of FMCD for one D: every window of D+1 consecutive sorted
 * sample keys, x[w] .. x[w+D], spans at least u(D). */
static int fmcd_windows_span(const double* x, uint64_t S, uint64_t D, double u) {
    for (uint64_t w = 0; w + D < S; ++w)
        if (!(x[w + D] - x[w] >= u)) return 0;
    return 1;
}

/* Fastest Minimum Conflict Degree on the sorted sample x[0..S), in fp64, from its definition
 * (Linear Models section): the conflict degree D is the smallest D >= 1 for which the window
 * condition above holds, searched over 1 <= D <= floor(S/3).  When no such D exists the
 * search gives up: D becomes floor(S/3) + 1 while the spread stays u(floor(S/3)) (the printed
 * procedure stops there with the spread of the last D it tried).  The model is then
 * a = 1/u and b = (K - a (x[S-1-D] + x[D])) / 2, which puts x[D] near t = 1 and x[S-1-D] near
 * t = K-1.
 *
 * The condition is monotone in D, also in fp64: a window's span x[w+D+1] - x[w] is at least
 * x[w+D] - x[w] (rounding is monotone), and u(D+1) <= u(D) because the trimmed range shrinks.
 * So the smallest D is found by bisection over [1, floor(S/3)], in O(S log S).
 * Returns 0, or -1 when S < 3 or K < 4. */
int oracle_fmcd(const double* x, uint64_t S, uint32_t K, double* a_out, double* b_out, uint64_t* D_out) {
    if (S < 3 || K < 4) return -1;
    const uint64_t Dmax = S / 3;
    uint64_t D;
    double u;
    if (!fmcd_windows_span(x, S, Dmax, fmcd_spread(x, S, Dmax, K))) {
        D = Dmax + 1;
        u = fmcd_spread(x, S, Dmax, K);
    } else {
        /* condition false below lo (or lo = 1), true at hi */
        uint64_t lo = 1, hi = Dmax;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (fmcd_windows_span(x, S, mid, fmcd_spread(x, S, mid, K)))
                hi = mid;
            else
                lo = mid + 1;
        }
        D = hi;
        u = fmcd_spread(x, S, D, K);
    }
    double a = 1.0 / u;
    double mid = x[S - 1 - D] + x[D];
    double am = a * mid;
    double b = ((double)K - am) / 2.0;
    *a_out = a;
    *b_out = b;
    *D_out = D;
    return 0;
}

/* ---------------------------------------------------------------- classification */

/* The clamped linear partition model of the Linear Models section, evaluated with one fp64
 * fused multiply-add.  Comparing t itself is the same as comparing floor(t): floor(t) < 0 iff
 * t < 0 and floor(t) >= K iff t >= K.  A NaN key (t is NaN) goes to the end its sign puts it. */
static uint32_t classify_linear(double a, double b, uint32_t K, double v, int neg) {
    double t = fma(a, v, b);
    if (t != t) return neg ? 0u : K - 1u;
    if (t < 0.0) return 0u;
    if (t >= (double)K) return K - 1u;
    return (uint32_t)t;
}

/* ---------------------------------------------------------------- two-level model (RMI section) */

/* Two-level piecewise-linear CDF model (a two-level RMI, F(x) = f2^(floor(M f1(x)))(x)):
 *   root   f1: FMCD fitted on the sorted sample onto M leaves, routed like classify_linear;
 *   leaf   l : t = min(max(fma(A_l, v, B_l), LO_l), HI_l), then clamped to [0, K) as above.
 * A leaf predicts K times the eCDF (the Machine Learning Models chapter: an eCDF model becomes
 * a partition model through floor(k F(x))).  Training targets of the sorted sample are
 * y_j = K (j + 1/2) / S.  Because the root is monotone, each leaf owns a contiguous index range
 * [first_l, first_l + cnt_l) of the sorted sample.  Each leaf is trained in its own centred
 * coordinate u = (v - c_l) / h_l (c_l the mean of its samples, h_l their largest distance to
 * it), as t = alpha_l u + beta_l. */
typedef struct {
    uint32_t M;
    double ra, rb;  /* root */
    double* leaf;   /* 4*M: A, B, LO, HI */
} l2pl_model;

static uint32_t l2pl_leaf(double ra, double rb, uint32_t M, double v) {
    return classify_linear(ra, rb, M, v, 0);
}

static uint32_t classify_l2pl(const l2pl_model* m, uint32_t K, double v, int neg) {
    if (v != v) return neg ? 0u : K - 1u;
    const double* q = m->leaf + 4 * (size_t)l2pl_leaf(m->ra, m->rb, m->M, v);
    double t = fma(q[0], v, q[1]);
    if (t < q[2]) t = q[2];
    if (t > q[3]) t = q[3];
    if (t < 0.0) return 0u;
    if (t >= (double)K) return K - 1u;
    return (uint32_t)t;
}

/* Sum of 64 partial sums in a fixed pairwise tree: partial p += partial p+s, s = 32, 16, ..., 1. */
static double tree_sum64(double* part) {
    for (int s = 32; s >= 1; s >>= 1)
        for (int p = 0; p < s; ++p) part[p] = part[p] + part[p + s];
    return part[0];
}

/* Leaf geometry of the sorted sample under the root (ra, rb): the index range of every leaf,
 * its centre c (mean of its samples), its scale h (largest |x - c|, or 1 when that is 0) and the
 * second moment m2 = mean of u^2 with u = (x - c) / h.  Sums use 64 strided partials (partial p
 * takes the leaf's samples p, p+64, ... in increasing order) and tree_sum64. */
void oracle_l2pl_geometry(const double* x, uint64_t S, uint32_t M, double ra, double rb, uint64_t* first /* M+1 */,
                          double* c, double* h, double* m2) {
    double part[64];
    for (uint32_t l = 0; l <= M; ++l) first[l] = 0;
    for (uint64_t j = 0; j < S; ++j) first[l2pl_leaf(ra, rb, M, x[j]) + 1] += 1;
    for (uint32_t l = 0; l < M; ++l) first[l + 1] += first[l];
    for (uint32_t l = 0; l < M; ++l) {
        uint64_t j0 = first[l], j1 = first[l + 1];
        c[l] = 0.0;
        h[l] = 1.0;
        m2[l] = 0.0;
        if (j1 == j0) continue;
        double cnt = (double)(j1 - j0);
        for (int p = 0; p < 64; ++p) part[p] = 0.0;
        for (uint64_t j = j0; j < j1; ++j) part[(j - j0) & 63] += x[j];
        double mean = tree_sum64(part) / cnt;
        double d0 = fabs(x[j0] - mean), d1 = fabs(x[j1 - 1] - mean);
        double scale = d0 > d1 ? d0 : d1;
        if (!(scale > 0.0)) scale = 1.0;
        for (int p = 0; p < 64; ++p) part[p] = 0.0;
        for (uint64_t j = j0; j < j1; ++j) {
            double u = (x[j] - mean) / scale;
            part[(j - j0) & 63] = fma(u, u, part[(j - j0) & 63]);
        }
        c[l] = mean;
        h[l] = scale;
        m2[l] = tree_sum64(part) / cnt;
    }
}

static double l2pl_target(uint64_t j, uint64_t S, uint32_t K) { return (double)K * ((double)j + 0.5) / (double)S; }

/* Forward and backward pass of every leaf's mean-squared error
 *   L_l = (1/cnt_l) sum_j (alpha_l u_j + beta_l - y_j)^2
 * at the given (alpha, beta) (2*M, interleaved).  grad (2*M) receives (dL/dalpha, dL/dbeta);
 * loss (M, nullable) receives L_l.  The sums run in a fixed order: 64 strided partials (partial
 * p takes the leaf's samples p, p+64, ... in increasing order, accumulated with fma for the
 * slope term), then tree_sum64. */
void oracle_l2pl_grad(const double* x, uint64_t S, uint32_t K, uint32_t M, const uint64_t* first, const double* c,
                      const double* h, const double* ab, double* grad, double* loss) {
    double pa[64], pb[64], pl[64];
    for (uint32_t l = 0; l < M; ++l) {
        uint64_t j0 = first[l], j1 = first[l + 1];
        for (int p = 0; p < 64; ++p) pa[p] = pb[p] = pl[p] = 0.0;
        for (uint64_t j = j0; j < j1; ++j) {
            int p = (int)((j - j0) & 63);
            double u = (x[j] - c[l]) / h[l];
            double r = fma(ab[2 * l], u, ab[2 * l + 1]) - l2pl_target(j, S, K);
            pa[p] = fma(r, u, pa[p]);
            pb[p] = pb[p] + r;
            pl[p] = fma(r, r, pl[p]);
        }
        uint64_t cnt = j1 - j0;
        double inv = cnt ? 2.0 / (double)cnt : 0.0;
        grad[2 * l] = tree_sum64(pa) * inv;
        grad[2 * l + 1] = tree_sum64(pb) * inv;
        if (loss) loss[l] = cnt ? tree_sum64(pl) / (double)cnt : 0.0;
    }
}

/* Training: root = FMCD onto M leaves; each leaf starts at the line through its first and last
 * sample (interpolation, the Learned Sort choice) and takes `iters` gradient steps.  With u
 * centred on the leaf mean the MSE's Hessian is diag(2 m2, 2), so the step is scaled per
 * coordinate by its inverse: alpha -= (1/2 / m2) g_alpha, beta -= g_beta / 2 (a Newton step,
 * which lands on the minimiser of the quadratic loss; later steps only absorb rounding and the
 * clamp).  The slope is kept >= 0 so the model stays monotone.  Export:
 * A = alpha / h, B = beta - A c; envelope LO_0 = 0, LO_l = HI_(l-1),
 * HI_l = max(LO_l, min(K, fma(A, last sample, B))) (an empty leaf has A = 0, B = LO_l = HI_l).
 * ab_out (2*M, nullable) receives the trained (alpha, beta).  Returns 0, or -1 when the root
 * fit fails or a coefficient is not finite. */
int oracle_l2pl_train(const double* x, uint64_t S, uint32_t K, uint32_t M, uint32_t iters, double* root_ab,
                      double* leaf_out, double* ab_out) {
    double ra, rb;
    uint64_t rD;
    if (oracle_fmcd(x, S, M, &ra, &rb, &rD) != 0) return -1;
    if (!(ra > 0.0) || !isfinite(ra) || !isfinite(rb)) return -1;
    uint64_t* first = (uint64_t*)malloc((M + 1) * sizeof(uint64_t));
    double* c = (double*)malloc(M * sizeof(double));
    double* h = (double*)malloc(M * sizeof(double));
    double* m2 = (double*)malloc(M * sizeof(double));
    double* ab = (double*)malloc(2 * (size_t)M * sizeof(double));
    double* g = (double*)malloc(2 * (size_t)M * sizeof(double));
    oracle_l2pl_geometry(x, S, M, ra, rb, first, c, h, m2);
    for (uint32_t l = 0; l < M; ++l) {
        uint64_t j0 = first[l], j1 = first[l + 1];
        double alpha = 0.0, beta = 0.0;
        if (j1 > j0) {
            double y0 = l2pl_target(j0, S, K), y1 = l2pl_target(j1 - 1, S, K);
            double u0 = (x[j0] - c[l]) / h[l], u1 = (x[j1 - 1] - c[l]) / h[l];
            if (u1 > u0) alpha = (y1 - y0) / (u1 - u0);
            beta = y0 - alpha * u0;
        }
        ab[2 * l] = alpha;
        ab[2 * l + 1] = beta;
    }
    for (uint32_t it = 0; it < iters; ++it) {
        oracle_l2pl_grad(x, S, K, M, first, c, h, ab, g, NULL);
        for (uint32_t l = 0; l < M; ++l) {
            if (first[l + 1] == first[l]) continue;
            double alpha = 0.0;
            if (m2[l] > 0.0) {
                double q = 0.5 / m2[l];
                alpha = ab[2 * l] - q * g[2 * l];
                if (!(alpha > 0.0)) alpha = 0.0;
            }
            ab[2 * l] = alpha;
            ab[2 * l + 1] = ab[2 * l + 1] - 0.5 * g[2 * l + 1];
        }
    }
    double prev_hi = 0.0;
    int ok = 1;
    for (uint32_t l = 0; l < M; ++l) {
        uint64_t j0 = first[l], j1 = first[l + 1];
        double A = 0.0, B = prev_hi, lo = prev_hi, hi = prev_hi;
        if (j1 > j0) {
            A = ab[2 * l] / h[l];
            B = ab[2 * l + 1] - A * c[l];
            double last = fma(A, x[j1 - 1], B);
            if (last > (double)K) last = (double)K;
            hi = last > lo ? last : lo;
        }
        if (!isfinite(A) || !isfinite(B) || !isfinite(hi)) ok = 0;
        leaf_out[4 * l + 0] = A;
        leaf_out[4 * l + 1] = B;
        leaf_out[4 * l + 2] = lo;
        leaf_out[4 * l + 3] = hi;
        prev_hi = hi;
    }
    if (ab_out) memcpy(ab_out, ab, 2 * (size_t)M * sizeof(double));
    root_ab[0] = ra;
    root_ab[1] = rb;
    free(first);
    free(c);
    free(h);
    free(m2);
    free(ab);
    free(g);
    return ok ? 0 : -1;
}

/* ---------------------------------------------------------------- one partition */

typedef struct {
    int dtype;
    const oracle_params* p;
    oracle_stats* st;
    size_t kb;
    char* aux_keys;
    uint32_t* aux_pay;
    uint32_t* bucket_of; /* scratch, n */
} ctx_t;

static uint32_t ilog2_floor(uint64_t v) {
    uint32_t r = 0;
    while (v >>= 1) ++r;
    return r;
}

static uint32_t bitlen(uint64_t v) {
    uint32_t r = 0;
    while (v) {
        ++r;
        v >>= 1;
    }
    return r;
}

/* Model of the bucket keys[0..n) whose first key sits at offset lo_rel of its array.
 * l2 receives the two-level model when it is chosen (its leaf array is owned by the caller). */
/* Splitter tree (the Decision Trees section: the comparison-based classifier of IPS4o, which the
 * paper's models are measured against).  Splitters are the sample quantiles
 * s_i = x[floor(i S / K)], i = 1 .. K-1, and a key goes to the number of splitters below it.  The
 * comparison is strict, except when every splitter equals the sample's largest value: then keys
 * equal to it must go past the splitters, or nothing would be split.  With at least two distinct
 * sample values the smallest and the largest sampled value always land in different buckets. */
static void fit_tree(const uint64_t* o, uint64_t S, uint32_t K, oracle_model* m) {
    m->kind = MODEL_TREE;
    m->degenerate = 0;
    for (uint32_t i = 1; i < K; ++i) m->split[i - 1] = o[((uint64_t)i * S) / K];
    m->tree_strict = m->split[0] < o[S - 1] ? 1u : 0u;
}

static uint32_t classify_tree(const oracle_model* m, uint64_t o) {
    uint32_t b = 0;
    for (uint32_t i = 0; i + 1 < m->K; ++i) b += (m->tree_strict ? m->split[i] < o : m->split[i] <= o) ? 1u : 0u;
    return b;
}

/* Equality buckets (IPS4o; applied to the linear model): a value whose run in the sorted sample
 * is longer than S/K (run * K > S) is heavy; at most min(16, (K-4)/2) of them, the smallest
 * first.  The linear part is fitted by FMCD on the sample without the heavy runs, with K - 2E
 * buckets; when that fit is unusable every other key goes to linear bucket 0.  A sample of one
 * value only (E = 1 and nothing else) is left to the degenerate handling (closure or digit split),
 * which guarantees progress.  Returns 1 when equality buckets are used (m filled). */
static int fit_equality(const double* x, const uint64_t* o, uint64_t S, uint32_t K, oracle_model* m) {
    uint32_t emax = (K - 4) / 2;
    if (emax > 16) emax = 16;
    uint32_t E = 0;
    uint64_t heavy_keys = 0;
    uint64_t run_lo[16], run_hi[16];
    for (uint64_t j = 0; j < S;) {
        uint64_t r = j;
        while (r < S && o[r] == o[j]) ++r;
        if ((r - j) * (uint64_t)K > S && E < emax) {
            m->heavy[E] = o[j];
            run_lo[E] = j;
            run_hi[E] = r;
            heavy_keys += r - j;
            ++E;
        }
        j = r;
    }
    if (E == 0 || (E == 1 && heavy_keys == S)) return 0;
    const uint64_t Sr = S - heavy_keys;
    double* xr = (double*)malloc((Sr ? Sr : 1) * sizeof(double));
    uint64_t q = 0;
    for (uint64_t j = 0, e = 0; j < S; ++j) {
        while (e < E && j >= run_hi[e]) ++e;
        if (e < E && j >= run_lo[e]) continue;  /* inside heavy run e */
        xr[q++] = x[j];
    }
    m->neq = E;
    m->Km = K - 2 * E;
    m->kind = MODEL_LINEAR;
    m->degenerate = 0;
    m->const0 = 1;
    if (Sr >= 3 && isfinite(xr[0]) && isfinite(xr[Sr - 1])) {
        double a, b;
        uint64_t D;
        if (oracle_fmcd(xr, Sr, m->Km, &a, &b, &D) == 0 && a > 0.0 && isfinite(a) && isfinite(b)) {
            m->a = a;
            m->b = b;
            m->D = D;
            m->const0 = 0;
        }
    }
    free(xr);
    return 1;
}

/* Buckets of the partition of a bucket of n keys.  IPLS keeps IPS4o's bucket count (Proposed
 * Algorithm), and IPS4o gives a subproblem close to the base case fewer buckets.  With
 * bucket_policy 1 and the plain FMCD line (model 0, no equality buckets, no inheritance) this
 * reading takes the smallest power of two k with k >= 8n/T (a bucket then expects at most T/8
 * keys), kept within [min(K, 64), K]; otherwise K. */
uint32_t oracle_bucket_count(uint64_t n, const oracle_params* p) {
    const uint32_t K = p->num_buckets;
    if (!p->bucket_policy || p->model != 0 || p->equality || p->inherit) return K;
    const uint64_t need = (8 * n + p->base_case_max - 1) / p->base_case_max;
    uint32_t k = 1;
    while (k < need && k < K) k <<= 1;
    const uint32_t lo = K < 64 ? K : 64;
    if (k < lo) k = lo;
    if (k > K) k = K;
    return k;
}

/* inh/inh_len: a sorted sample handed down by the parent (sample inheritance), used instead of a
 * fresh one.  sample_out (nullable): receives the sorted sample's ords (caller frees).  adapt: the
 * bucket count follows oracle_bucket_count (a bucket of the recursion); else K (one pass of the
 * whole array, as asked). */
static void fit_bucket(const void* keys, uint64_t n, int dtype, const oracle_params* p_in, uint64_t lo_rel,
                       oracle_model* m, l2pl_model* l2, double* l2_leaf, const uint64_t* inh, uint64_t inh_len,
                       uint64_t** sample_out, uint64_t* sample_len, int adapt) {
    /* the sample size's 2K minimum (and the paper's alpha K - 1) follow the bucket's K */
    oracle_params q = *p_in;
    if (adapt) q.num_buckets = oracle_bucket_count(n, p_in);
    const oracle_params* p = &q;
    uint32_t K = p->num_buckets;
    memset(m, 0, sizeof(*m));
    m->K = K;
    uint64_t S = inh_len ? inh_len : oracle_sample_size(n, p);
    m->S = S;
    double* x = (double*)malloc((S ? S : 1) * sizeof(double));
    uint64_t* o = (uint64_t*)malloc((S ? S : 1) * sizeof(uint64_t));
    if (inh_len) {
        memcpy(o, inh, S * sizeof(uint64_t));
        for (uint64_t j = 0; j < S; ++j) x[j] = val_from_ord(o[j], dtype);
    } else {
        sorted_sample_ords(keys, n, dtype, lo_rel, S, p->seed, x, o);
    }
    if (sample_out) {
        *sample_out = (uint64_t*)malloc((S ? S : 1) * sizeof(uint64_t));
        memcpy(*sample_out, o, S * sizeof(uint64_t));
        *sample_len = S;
    }
    if (p->model == 3 && S >= 1 && o[0] != o[S - 1]) {
        fit_tree(o, S, K, m);
        free(x);
        free(o);
        return;
    }
    if (p->equality && fit_equality(x, o, S, K, m)) {
        free(x);
        free(o);
        return;
    }
    free(o);
    int degenerate = 1;
    if (S >= 3 && isfinite(x[0]) && isfinite(x[S - 1])) {
        double a, b;
        uint64_t D;
        if (oracle_fmcd(x, S, K, &a, &b, &D) == 0) {
            m->a = a;
            m->b = b;
            m->D = D;
            degenerate = !(a > 0.0) || !isfinite(a) || !isfinite(b);
        }
    }
    m->degenerate = (uint32_t)degenerate;
    if (degenerate) {
        uint64_t umin = UINT64_MAX, umax = 0;
        for (uint64_t i = 0; i < n; ++i) {
            uint64_t o = oracle_ord_one(keys, i, dtype);
            if (o < umin) umin = o;
            if (o > umax) umax = o;
        }
        if (umin == umax) {
            m->kind = MODEL_CLOSED;
        } else {
            int sh = (int)bitlen(umax - umin) - (int)ilog2_floor(K);
            m->kind = MODEL_MSD;
            m->umin = umin;
            m->shift = (uint32_t)(sh > 0 ? sh : 0);
        }
        free(x);
        return;
    }
    m->kind = MODEL_LINEAR;
    /* Every D + 1 consecutive sample keys span at least a bucket's width, so a bucket of the line
     * holds at most about D of the S sample keys, D n / S of the bucket's n.  The auto policy tries
     * the two-level model only where that can exceed the base-case threshold T (D n > T S, in
     * integers as D > floor(T S / n)): elsewhere FMCD already leaves no bucket for another level. */
    const int try_l2pl = p->model == 2 || (p->model == 1 && m->D > (uint64_t)p->base_case_max * S / n);
    if (p->model != 0 && try_l2pl && l2 && l2_leaf) {
        double root[2];
        l2->M = p->leaves ? p->leaves : 256;
        l2->leaf = l2_leaf;
        if (oracle_l2pl_train(x, S, K, l2->M, p->train_iters, root, l2_leaf, NULL) == 0) {
            l2->ra = root[0];
            l2->rb = root[1];
            /* max sample load under each model; the two-level model replaces FMCD only when
             * its max load is strictly lower (or always, when forced) */
            uint64_t* h1 = (uint64_t*)calloc(K, sizeof(uint64_t));
            uint64_t* h2 = (uint64_t*)calloc(K, sizeof(uint64_t));
            for (uint64_t j = 0; j < S; ++j) {
                h1[classify_linear(m->a, m->b, K, x[j], 0)] += 1;
                h2[classify_l2pl(l2, K, x[j], 0)] += 1;
            }
            uint64_t m1 = 0, m2 = 0;
            for (uint32_t c = 0; c < K; ++c) {
                if (h1[c] > m1) m1 = h1[c];
                if (h2[c] > m2) m2 = h2[c];
            }
            m->max_load_linear = m1;
            m->max_load_l2pl = m2;
            /* a forced or chosen two-level model must still split the sample, or the recursion
             * would not progress */
            int splits = m2 < S;
            if (splits && (p->model == 2 || m2 < m1)) m->kind = MODEL_L2PL;
            free(h1);
            free(h2);
        }
    }
    free(x);
}

/* Equality buckets (IPS4o's, for keys repeated often in the sample): with heavy values
 * h_0 < ... < h_(E-1) the linear part has K - 2E buckets, and a key goes to
 *   linear bucket + 2 * #{e : h_e < key} + [key is some h_e],
 * which keeps the buckets in key order: each heavy value gets a bucket of its own between the
 * keys below it and the keys above it.  Such a bucket holds one value only, so the recursion
 * closes it where it is made (it counts as closed, and is neither partitioned nor base-sorted). */
static uint32_t classify_equality(const oracle_model* m, uint64_t o, double v, int neg) {
    uint32_t less = 0, eq = 0;
    for (uint32_t e = 0; e < m->neq; ++e) {
        less += m->heavy[e] < o ? 1u : 0u;
        eq |= m->heavy[e] == o ? 1u : 0u;
    }
    uint32_t b = m->const0 ? 0u : classify_linear(m->a, m->b, m->Km, v, neg);
    return b + 2u * less + eq;
}

static uint32_t classify_key(const void* keys, uint64_t i, int dtype, const oracle_model* m, const l2pl_model* l2) {
    if (m->kind == MODEL_MSD) return (uint32_t)((oracle_ord_one(keys, i, dtype) - m->umin) >> m->shift);
    if (m->kind == MODEL_TREE) return classify_tree(m, oracle_ord_one(keys, i, dtype));
    double v = oracle_val_one(keys, i, dtype);
    int neg = key_negative(keys, i, dtype);
    if (m->kind == MODEL_L2PL) return classify_l2pl(l2, m->K, v, neg);
    if (m->neq) return classify_equality(m, oracle_ord_one(keys, i, dtype), v, neg);
    return classify_linear(m->a, m->b, m->K, v, neg);
}

/* Stable distribution of keys[0..n) (and payload) into contiguous buckets: count, exclusive
 * prefix, then move each key, in index order, to the next free slot of its bucket. */
static void distribute(ctx_t* cx, char* keys, uint32_t* pay, uint64_t n, const oracle_model* m,
                       const l2pl_model* l2, uint64_t* counts) {
    uint32_t K = m->K;
    size_t kb = cx->kb;
    uint64_t* next = (uint64_t*)calloc(K, sizeof(uint64_t));
    for (uint32_t c = 0; c < K; ++c) counts[c] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t c = classify_key(keys, i, cx->dtype, m, l2);
        cx->bucket_of[i] = c;
        counts[c] += 1;
    }
    uint64_t run = 0;
    for (uint32_t c = 0; c < K; ++c) {
        next[c] = run;
        run += counts[c];
    }
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t d = next[cx->bucket_of[i]]++;
        memcpy(cx->aux_keys + d * kb, keys + i * kb, kb);
        if (pay) cx->aux_pay[d] = pay[i];
    }
    memcpy(keys, cx->aux_keys, n * kb);
    if (pay) memcpy(pay, cx->aux_pay, n * sizeof(uint32_t));
    free(next);
}

/* ---------------------------------------------------------------- base case */

/* Stable sort by ord of keys[0..n) (and payload): a plain top-down merge sort on (ord, index). */
typedef struct {
    uint64_t ord;
    uint64_t idx;
} ordidx;

static void merge_sort_oi(ordidx* a, ordidx* tmp, uint64_t n) {
    if (n < 2) return;
    uint64_t h = n / 2;
    merge_sort_oi(a, tmp, h);
    merge_sort_oi(a + h, tmp, n - h);
    uint64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        if (a[j].ord < a[i].ord) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, n * sizeof(ordidx));
}

static void base_case(ctx_t* cx, char* keys, uint32_t* pay, uint64_t n) {
    if (n < 2) return;
    size_t kb = cx->kb;
    ordidx* a = (ordidx*)malloc(n * sizeof(ordidx));
    ordidx* t = (ordidx*)malloc(n * sizeof(ordidx));
    for (uint64_t i = 0; i < n; ++i) {
        a[i].ord = oracle_ord_one(keys, i, cx->dtype);
        a[i].idx = i;
    }
    merge_sort_oi(a, t, n);
    for (uint64_t i = 0; i < n; ++i) {
        memcpy(cx->aux_keys + i * kb, keys + a[i].idx * kb, kb);
        if (pay) cx->aux_pay[i] = pay[a[i].idx];
    }
    memcpy(keys, cx->aux_keys, n * kb);
    if (pay) memcpy(pay, cx->aux_pay, n * sizeof(uint32_t));
    free(a);
    free(t);
    cx->st->base_cases += 1;
}

/* ---------------------------------------------------------------- sample inheritance */

/* The raw key whose ord is o (inverse of the key map). */
static void key_from_ord(uint64_t o, int dtype, unsigned char* buf) {
    if (dtype == OR_U64) {
        memcpy(buf, &o, 8);
    } else if (dtype == OR_F32) {
        uint32_t u = (uint32_t)o;
        u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
        memcpy(buf, &u, 4);
    } else {
        uint64_t u = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
        memcpy(buf, &u, 8);
    }
}

/* Smallest inherited sample that is used: sample_min (0 means 2K), and at least 3 (FMCD's own
 * minimum). */
static uint64_t inherit_min(const oracle_params* p) {
    uint64_t t = p->sample_min ? p->sample_min : 2ull * p->num_buckets;
    return t < 3 ? 3 : t;
}

/* Whether FMCD on the sorted sample o[0..S) gives a usable line: the test fit_bucket applies
 * before it falls back to the degenerate rule. */
static int fmcd_usable(const uint64_t* o, uint64_t S, int dtype, uint32_t K) {
    if (S < 3) return 0;
    double* x = (double*)malloc(S * sizeof(double));
    for (uint64_t j = 0; j < S; ++j) x[j] = val_from_ord(o[j], dtype);
    int ok = 0;
    if (isfinite(x[0]) && isfinite(x[S - 1])) {
        double a, b;
        uint64_t D;
        ok = oracle_fmcd(x, S, K, &a, &b, &D) == 0 && a > 0.0 && isfinite(a) && isfinite(b);
    }
    free(x);
    return ok;
}

/* The parent's sorted sample smp[0..slen) split by the parent's model: the sample keys of child c,
 * in their sorted order, are (*sub)[(*sub_off)[c] .. (*sub_off)[c+1]) (caller frees both). */
static void restrict_sample(const uint64_t* smp, uint64_t slen, int dtype, const oracle_model* m,
                            const l2pl_model* l2, uint64_t** sub, uint64_t** sub_off) {
    const uint32_t K = m->K;
    *sub = (uint64_t*)malloc((slen ? slen : 1) * sizeof(uint64_t));
    *sub_off = (uint64_t*)calloc((size_t)K + 1, sizeof(uint64_t));
    uint32_t* cls = (uint32_t*)malloc((slen ? slen : 1) * sizeof(uint32_t));
    unsigned char kbuf[8];
    for (uint64_t j = 0; j < slen; ++j) {
        key_from_ord(smp[j], dtype, kbuf);
        cls[j] = classify_key(kbuf, 0, dtype, m, l2);
        (*sub_off)[cls[j] + 1] += 1;
    }
    for (uint32_t c = 0; c < K; ++c) (*sub_off)[c + 1] += (*sub_off)[c];
    uint64_t* fill = (uint64_t*)malloc((size_t)K * sizeof(uint64_t));
    memcpy(fill, *sub_off, (size_t)K * sizeof(uint64_t));
    for (uint64_t j = 0; j < slen; ++j) (*sub)[fill[cls[j]]++] = smp[j];
    free(fill);
    free(cls);
}

/* Whether a child of n keys inherits the restricted sample r[0..len). */
static int child_inherits(const oracle_params* p, uint64_t n, const uint64_t* r, uint64_t len, int dtype) {
    return n > p->base_case_max && len >= inherit_min(p) && fmcd_usable(r, len, dtype, p->num_buckets);
}

/* ---------------------------------------------------------------- recursion (Proposed Algorithm) */

/* inh/inh_len: the bucket's inherited sorted sample (ords), or NULL/0 for a fresh sample.
 * With inherit on, a child of a bucket partitioned by the FMCD line inherits the parent's sorted
 * sample restricted to the child (the sample keys the line sends there, still sorted) when the
 * child is partitioned itself (more than T keys), the restricted sample holds at least
 * inherit_min keys and FMCD on it is usable; every other bucket draws a fresh sample. */
static void ipls(ctx_t* cx, char* keys, uint32_t* pay, uint64_t n, uint64_t lo_rel, uint64_t level,
                 const uint64_t* inh, uint64_t inh_len) {
    const oracle_params* p = cx->p;
    if (n <= p->base_case_max) {
        base_case(cx, keys, pay, n);
        return;
    }
    oracle_model m;
    l2pl_model l2 = {0, 0.0, 0.0, NULL};
    uint32_t M = p->leaves ? p->leaves : 256;
    double* leaf = p->model ? (double*)malloc(4 * (size_t)M * sizeof(double)) : NULL;
    uint64_t* smp = NULL;
    uint64_t slen = 0;
    fit_bucket(keys, n, cx->dtype, p, lo_rel, &m, &l2, leaf, inh, inh_len, p->inherit ? &smp : NULL, &slen, 1);
    if (m.kind == MODEL_CLOSED) {
        cx->st->closed += 1;
        free(leaf);
        free(smp);
        return;
    }
    if (m.kind == MODEL_MSD) cx->st->fallback += 1;
    if (m.kind == MODEL_L2PL) cx->st->l2pl_used += 1;
    if (inh_len) cx->st->inherited += 1;
    cx->st->passes += 1;
    cx->st->keys_partitioned += n;
    if (level > cx->st->max_level) cx->st->max_level = level;
    uint32_t K = m.K;
    uint64_t* counts = (uint64_t*)malloc(K * sizeof(uint64_t));
    distribute(cx, keys, pay, n, &m, &l2, counts);
    free(leaf);
    if (level == 1) {
        uint64_t mx = 0;
        for (uint32_t c = 0; c < K; ++c)
            if (counts[c] > mx) mx = counts[c];
        cx->st->level1_max_load = mx;
    }
    uint64_t* sub = NULL;
    uint64_t* sub_off = NULL;
    if (smp && m.kind == MODEL_LINEAR && m.neq == 0) restrict_sample(smp, slen, cx->dtype, &m, &l2, &sub, &sub_off);
    free(smp);
    /* an equality bucket holds one value only: it is closed where it is made */
    uint32_t eqb[16];
    const uint32_t neq = m.kind == MODEL_LINEAR ? m.neq : 0;
    for (uint32_t e = 0; e < neq; ++e) {
        const uint64_t o = m.heavy[e];
        const int neg = cx->dtype == OR_U64 ? 0 : (cx->dtype == OR_F32 ? !((o >> 31) & 1u) : !(o >> 63));
        eqb[e] = classify_equality(&m, o, val_from_ord(o, cx->dtype), neg);
    }
    uint64_t off = 0;
    for (uint32_t c = 0; c < K; ++c) {
        uint64_t cnt = counts[c];
        int is_eq = 0;
        for (uint32_t e = 0; e < neq; ++e) is_eq |= eqb[e] == c;
        if (cnt > 0 && is_eq) {
            cx->st->closed += 1;
        } else if (cnt > 0) {
            const uint64_t* ci = NULL;
            uint64_t cl = 0;
            if (sub && child_inherits(p, cnt, sub + sub_off[c], sub_off[c + 1] - sub_off[c], cx->dtype)) {
                ci = sub + sub_off[c];
                cl = sub_off[c + 1] - sub_off[c];
            }
            ipls(cx, keys + off * cx->kb, pay ? pay + off : NULL, cnt, lo_rel + off, level + 1, ci, cl);
        }
        off += cnt;
    }
    free(sub);
    free(sub_off);
    free(counts);
}

/* Sample inheritance is defined for the FMCD line alone (no two-level model, splitter tree or
 * equality buckets). */
static int params_ok(const oracle_params* p) {
    return p && p->num_buckets >= 4 && p->base_case_max >= 1 && p->inherit <= 1 &&
           (!p->inherit || (p->model == 0 && !p->equality));
}

static int ctx_init(ctx_t* cx, int dtype, const oracle_params* p, oracle_stats* st, uint64_t n, int has_pay) {
    cx->dtype = dtype;
    cx->p = p;
    cx->st = st;
    cx->kb = key_bytes(dtype);
    cx->aux_keys = (char*)malloc((n ? n : 1) * cx->kb);
    cx->aux_pay = has_pay ? (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t)) : NULL;
    cx->bucket_of = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    return cx->aux_keys && cx->bucket_of && (!has_pay || cx->aux_pay);
}

static void ctx_free(ctx_t* cx) {
    free(cx->aux_keys);
    free(cx->aux_pay);
    free(cx->bucket_of);
}

/* Sort keys[0..n) (and payload) in place.  Returns 0, or -1 on bad arguments. */
int oracle_sort(void* keys, uint32_t* payload, uint64_t n, int dtype, const oracle_params* p, oracle_stats* st) {
    if (!params_ok(p) || dtype < 0 || dtype > 2) return -1;
    oracle_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    if (n < 2) return 0;
    ctx_t cx;
    if (!ctx_init(&cx, dtype, p, st, n, payload != NULL)) {
        ctx_free(&cx);
        return -1;
    }
    ipls(&cx, (char*)keys, payload, n, 0, 1, NULL, 0);
    ctx_free(&cx);
    return 0;
}

/* Sort every segment [off[s], off[s+1]) independently; sample offsets are relative to each
 * segment's start, so a segment sorts exactly as it would alone. */
int oracle_sort_segmented(void* keys, uint32_t* payload, const uint64_t* off, uint64_t nseg, int dtype,
                          const oracle_params* p, oracle_stats* st) {
    if (!params_ok(p)) return -1;
    oracle_stats acc;
    memset(&acc, 0, sizeof(acc));
    size_t kb = key_bytes(dtype);
    for (uint64_t s = 0; s < nseg; ++s) {
        if (off[s + 1] < off[s]) return -1;
        oracle_stats one;
        int rc = oracle_sort((char*)keys + off[s] * kb, payload ? payload + off[s] : NULL, off[s + 1] - off[s],
                             dtype, p, &one);
        if (rc) return rc;
        acc.passes += one.passes;
        acc.closed += one.closed;
        acc.fallback += one.fallback;
        acc.base_cases += one.base_cases;
        acc.l2pl_used += one.l2pl_used;
        acc.keys_partitioned += one.keys_partitioned;
        acc.inherited += one.inherited;
        if (one.max_level > acc.max_level) acc.max_level = one.max_level;
        if (one.level1_max_load > acc.level1_max_load) acc.level1_max_load = one.level1_max_load;
    }
    if (st) *st = acc;
    return 0;
}

/* The model a bucket of n keys at offset lo_rel gets (sample, sort, fit, degenerate handling).
 * When the two-level model is chosen, leaf_out (4*M doubles) and root_out (2) receive it. */
int oracle_fit_bucket(const void* keys, uint64_t n, int dtype, const oracle_params* p, uint64_t lo_rel,
                      oracle_model* m, double* root_out, double* leaf_out) {
    if (!params_ok(p) || n < 2) return -1;
    uint32_t M = p->leaves ? p->leaves : 256;
    l2pl_model l2 = {0, 0.0, 0.0, NULL};
    double* leaf = p->model ? (double*)malloc(4 * (size_t)M * sizeof(double)) : NULL;
    fit_bucket(keys, n, dtype, p, lo_rel, m, &l2, leaf, NULL, 0, NULL, NULL, 1);
    if (m->kind == MODEL_L2PL && leaf_out && root_out) {
        memcpy(leaf_out, leaf, 4 * (size_t)M * sizeof(double));
        root_out[0] = l2.ra;
        root_out[1] = l2.rb;
    }
    free(leaf);
    return 0;
}

/* The sorted sample (ords) that bucket c of the first level inherits, into out (room for the
 * level's sample size); *len = 0 when it draws a fresh one.  Returns 0, or -1 on bad arguments. */
int oracle_child_sample(const void* keys, uint64_t n, int dtype, const oracle_params* p, uint32_t c, uint64_t* out,
                        uint64_t* len) {
    *len = 0;
    if (!params_ok(p) || !p->inherit || n < 2 || c >= p->num_buckets) return -1;
    oracle_model m;
    uint64_t* smp = NULL;
    uint64_t slen = 0;
    fit_bucket(keys, n, dtype, p, 0, &m, NULL, NULL, NULL, 0, &smp, &slen, 1);
    if (m.kind == MODEL_LINEAR && m.neq == 0 && n > p->base_case_max) {
        uint64_t* sub = NULL;
        uint64_t* sub_off = NULL;
        restrict_sample(smp, slen, dtype, &m, NULL, &sub, &sub_off);
        uint64_t cnt = 0;
        for (uint64_t i = 0; i < n; ++i) cnt += classify_key(keys, i, dtype, &m, NULL) == c;
        const uint64_t l = sub_off[c + 1] - sub_off[c];
        if (child_inherits(p, cnt, sub + sub_off[c], l, dtype)) {
            memcpy(out, sub + sub_off[c], l * sizeof(uint64_t));
            *len = l;
        }
        free(sub);
        free(sub_off);
    }
    free(smp);
    return 0;
}

/* One distribution pass over the whole array (level 1 only): fit, classify, stable scatter.
 * counts receives K bucket sizes (all zero when the bucket was closed).  Returns 0. */
int oracle_partition(void* keys, uint32_t* payload, uint64_t n, int dtype, const oracle_params* p,
                     oracle_model* m_out, uint64_t* counts) {
    if (!params_ok(p) || n < 2) return -1;
    oracle_stats st;
    memset(&st, 0, sizeof(st));
    ctx_t cx;
    if (!ctx_init(&cx, dtype, p, &st, n, payload != NULL)) {
        ctx_free(&cx);
        return -1;
    }
    uint32_t M = p->leaves ? p->leaves : 256;
    l2pl_model l2 = {0, 0.0, 0.0, NULL};
    double* leaf = p->model ? (double*)malloc(4 * (size_t)M * sizeof(double)) : NULL;
    oracle_model m;
    fit_bucket(keys, n, dtype, p, 0, &m, &l2, leaf, NULL, 0, NULL, NULL, 0);
    for (uint32_t c = 0; c < p->num_buckets; ++c) counts[c] = 0;
    if (m.kind != MODEL_CLOSED) distribute(&cx, (char*)keys, payload, n, &m, &l2, counts);
    if (m_out) *m_out = m;
    free(leaf);
    ctx_free(&cx);
    return 0;
}

/* Bucket of every key under a given linear model (used with the Worked Example's a, b). */
void oracle_classify_linear(const void* keys, uint64_t n, int dtype, double a, double b, uint32_t K,
                            uint32_t* out) {
    for (uint64_t i = 0; i < n; ++i)
        out[i] = classify_linear(a, b, K, oracle_val_one(keys, i, dtype), key_negative(keys, i, dtype));
}

/* Bucket of every key under a fitted model (any kind). */
void oracle_classify_model(const void* keys, uint64_t n, int dtype, const oracle_model* m, const double* root,
                           const double* leaf, uint32_t M, uint32_t* out) {
    l2pl_model l2 = {M, root ? root[0] : 0.0, root ? root[1] : 0.0, (double*)leaf};
    for (uint64_t i = 0; i < n; ++i) out[i] = classify_key(keys, i, dtype, m, &l2);
}

/* Stable distribution by a given bucket vector (counting-sort layout). */
void oracle_stable_layout(const void* keys, uint64_t n, int dtype, const uint32_t* bucket, uint32_t K, void* out) {
    size_t kb = key_bytes(dtype);
    uint64_t* next = (uint64_t*)calloc(K, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) next[bucket[i]] += 1;
    uint64_t run = 0;
    for (uint32_t c = 0; c < K; ++c) {
        uint64_t t = next[c];
        next[c] = run;
        run += t;
    }
    for (uint64_t i = 0; i < n; ++i)
        memcpy((char*)out + (next[bucket[i]]++) * kb, (const char*)keys + i * kb, kb);
    free(next);
}

/* IPS4o's buffered distribution (Background, IPS4o section; Worked Example): keys go, in
 * index order, into per-bucket buffers of b keys; a full buffer is flushed to the next free
 * block of the array; at the end the partial buffers are appended in bucket order.  Only the
 * Worked Example's intermediate layout uses it. */
void oracle_buffered_layout(const void* keys, uint64_t n, int dtype, const uint32_t* bucket, uint32_t K,
                            uint32_t bsize, void* out) {
    size_t kb = key_bytes(dtype);
    char* buf = (char*)malloc((size_t)K * bsize * kb);
    uint32_t* fill = (uint32_t*)calloc(K, sizeof(uint32_t));
    uint64_t w = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t c = bucket[i];
        memcpy(buf + ((size_t)c * bsize + fill[c]) * kb, (const char*)keys + i * kb, kb);
        if (++fill[c] == bsize) {
            memcpy((char*)out + w * kb, buf + (size_t)c * bsize * kb, (size_t)bsize * kb);
            w += bsize;
            fill[c] = 0;
        }
    }
    for (uint32_t c = 0; c < K; ++c) {
        memcpy((char*)out + w * kb, buf + (size_t)c * bsize * kb, (size_t)fill[c] * kb);
        w += fill[c];
    }
    free(buf);
    free(fill);
}
