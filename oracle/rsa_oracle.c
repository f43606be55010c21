/*
 * Plain CPU oracle for batched RSA modular exponentiation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * measured against; it is compiled into its own shared object and is loaded
 * only by the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark.  It shares no source, header, table or helper with the GPU
 * library, and the GPU library never calls it.
 *
 * What it computes is the plain definition of RSA encryption and decryption,
 * C = M^e mod n and M = C^d mod n (paper, Section 2 and Sections 3.2-3.3),
 * with no Montgomery form, no windowing and no Chinese remaindering:
 *
 *   - numbers are little-endian arrays of 32-bit limbs (limb 0 least
 *     significant), handled as (pointer, length) spans;
 *   - multiplication is the schoolbook method (Knuth, TAOCP vol. 2,
 *     Section 4.3.1, Algorithm M);
 *   - reduction is long division (Knuth, TAOCP vol. 2, Section 4.3.1,
 *     Algorithm D), keeping the remainder;
 *   - a modular product is a full product followed by a reduction, which is
 *     the product rule of the paper's modular-arithmetic identities (Fig. 3);
 *   - exponentiation is the left-to-right binary square-and-multiply method
 *     (paper, Section 3.6.3, Fig. 5, second algorithm), after reducing the
 *     base modulo n as the paper's device routine does first (Algorithm 2).
 *
 * Two further methods are test-only cross-checks: the naive repeated
 * multiplication of Section 3.6.2 (Fig. 4) and the right-to-left binary
 * method of Section 3.6.3 (Fig. 5, first algorithm).
 *
 * Conventions where the paper is silent: x^0 mod n = 1 mod n (so 0 when
 * n = 1), and a base at or above n is reduced first.  A zero modulus is an
 * error (status -1); the oracle accepts any modulus >= 1, odd or even.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <time.h>

typedef uint32_t limb_t;
typedef uint64_t dlimb_t;

/* ---- spans ------------------------------------------------------------- */

/* Length of x once leading zero limbs are dropped. */
static int bn_len(const limb_t *x, int n)
{
    while (n > 0 && x[n - 1] == 0) --n;
    return n;
}

/* -1, 0, +1 as a <, =, > b (both normalised). */
static int bn_cmp(const limb_t *a, int an, const limb_t *b, int bn)
{
    if (an != bn) return an < bn ? -1 : 1;
    for (int i = an - 1; i >= 0; --i)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

/* ---- Algorithm M: w[0 .. m+n-1] = u[0 .. m-1] * v[0 .. n-1] ------------ */
void oracle_bn_mul(limb_t *w, const limb_t *u, int m, const limb_t *v, int n)
{
    for (int i = 0; i < m + n; ++i) w[i] = 0;
    for (int j = 0; j < n; ++j) {
        dlimb_t k = 0;
        for (int i = 0; i < m; ++i) {
            dlimb_t t = (dlimb_t)u[i] * v[j] + w[i + j] + k;
            w[i + j] = (limb_t)t;
            k = t >> 32;
        }
        w[j + m] = (limb_t)k;
    }
}

/* ---- Algorithm D, remainder only ----------------------------------------
 * r[0 .. vn-1] = u mod v, where u has un limbs and v has vn limbs.
 * Requires v != 0.  Scratch: two arrays supplied by the caller of at least
 * un+1 and vn limbs.  Leading zero limbs in u or v are allowed.
 */
static void bn_mod_knuth(limb_t *r, const limb_t *u, int un, const limb_t *v, int vn,
                         limb_t *uwork, limb_t *vwork)
{
    int n = bn_len(v, vn);
    int ul = bn_len(u, un);
    for (int i = 0; i < vn; ++i) r[i] = 0;
    if (bn_cmp(u, ul, v, n) < 0) {           /* u < v: remainder is u */
        for (int i = 0; i < ul; ++i) r[i] = u[i];
        return;
    }
    if (n == 1) {                             /* short division */
        dlimb_t rem = 0;
        for (int i = ul - 1; i >= 0; --i)
            rem = ((rem << 32) | u[i]) % v[0];
        r[0] = (limb_t)rem;
        return;
    }
    int m = ul - n;                           /* quotient has m+1 limbs */

    /* D1: normalise so the divisor's top bit is set. */
    int s = __builtin_clz(v[n - 1]);
    for (int i = n - 1; i > 0; --i)
        vwork[i] = s ? (v[i] << s) | (v[i - 1] >> (32 - s)) : v[i];
    vwork[0] = v[0] << s;
    uwork[ul] = s ? u[ul - 1] >> (32 - s) : 0;
    for (int i = ul - 1; i > 0; --i)
        uwork[i] = s ? (u[i] << s) | (u[i - 1] >> (32 - s)) : u[i];
    uwork[0] = u[0] << s;

    const dlimb_t B = (dlimb_t)1 << 32;
    /* D2..D7: one quotient digit per step, most significant first. */
    for (int j = m; j >= 0; --j) {
        /* D3: estimate qhat from the top two limbs, then correct it. */
        dlimb_t num = ((dlimb_t)uwork[j + n] << 32) | uwork[j + n - 1];
        dlimb_t qhat = num / vwork[n - 1];
        dlimb_t rhat = num % vwork[n - 1];
        while (qhat >= B ||
               qhat * vwork[n - 2] > ((rhat << 32) | uwork[j + n - 2])) {
            qhat -= 1;
            rhat += vwork[n - 1];
            if (rhat >= B) break;
        }
        /* D4: multiply and subtract qhat * v from u[j .. j+n]. */
        int64_t borrow = 0;
        dlimb_t carry = 0;
        for (int i = 0; i < n; ++i) {
            dlimb_t p = qhat * vwork[i] + carry;
            carry = p >> 32;
            int64_t t = (int64_t)uwork[i + j] - (int64_t)(limb_t)p + borrow;
            uwork[i + j] = (limb_t)t;
            borrow = t >> 32;                 /* 0 or -1 */
        }
        int64_t t = (int64_t)uwork[j + n] - (int64_t)carry + borrow;
        uwork[j + n] = (limb_t)t;
        /* D5/D6: if the result went negative, qhat was one too large:
         * add the divisor back once. */
        if (t < 0) {
            dlimb_t c = 0;
            for (int i = 0; i < n; ++i) {
                dlimb_t sum = (dlimb_t)uwork[i + j] + vwork[i] + c;
                uwork[i + j] = (limb_t)sum;
                c = sum >> 32;
            }
            uwork[j + n] += (limb_t)c;
        }
    }
    /* D8: un-normalise the remainder. */
    for (int i = 0; i < n - 1; ++i)
        r[i] = s ? (uwork[i] >> s) | (uwork[i + 1] << (32 - s)) : uwork[i];
    r[n - 1] = uwork[n - 1] >> s;
}

/* Bit-serial shift-and-subtract remainder: slow, used only to cross-check
 * Algorithm D in the tests.  r has vn limbs; tmp has vn+1 limbs. */
static void bn_mod_shift_subtract(limb_t *r, const limb_t *u, int un, const limb_t *v, int vn,
                                  limb_t *tmp)
{
    for (int i = 0; i <= vn; ++i) tmp[i] = 0;
    for (int bit = un * 32 - 1; bit >= 0; --bit) {
        /* tmp = 2*tmp + bit */
        limb_t in = (u[bit / 32] >> (bit % 32)) & 1u;
        for (int i = 0; i <= vn; ++i) {
            limb_t out = tmp[i] >> 31;
            tmp[i] = (tmp[i] << 1) | in;
            in = out;
        }
        /* if tmp >= v: tmp -= v */
        int ge = 1;
        if (tmp[vn] == 0) {
            for (int i = vn - 1; i >= 0; --i) {
                if (tmp[i] != v[i]) { ge = tmp[i] > v[i]; break; }
            }
        }
        if (ge) {
            int64_t borrow = 0;
            for (int i = 0; i < vn; ++i) {
                int64_t t = (int64_t)tmp[i] - v[i] + borrow;
                tmp[i] = (limb_t)t;
                borrow = t >> 32;
            }
            tmp[vn] = (limb_t)((int64_t)tmp[vn] + borrow);
        }
    }
    for (int i = 0; i < vn; ++i) r[i] = tmp[i];
}

/* ---- modular product (Fig. 3 product rule) ------------------------------ */

typedef struct {
    int k;           /* limb width of every residue */
    limb_t *prod;    /* 2k   */
    limb_t *uwork;   /* 2k+1 */
    limb_t *vwork;   /* k    */
} ctx_t;

static int ctx_init(ctx_t *c, int k)
{
    c->k = k;
    c->prod = (limb_t *)malloc(sizeof(limb_t) * (size_t)(2 * k + 2));
    c->uwork = (limb_t *)malloc(sizeof(limb_t) * (size_t)(2 * k + 2));
    c->vwork = (limb_t *)malloc(sizeof(limb_t) * (size_t)(k + 1));
    return (c->prod && c->uwork && c->vwork) ? 0 : -1;
}

static void ctx_free(ctx_t *c)
{
    free(c->prod); free(c->uwork); free(c->vwork);
}

/* r = a*b mod n; a, b, r, n all k limbs; r may alias a or b. */
static void modmul(ctx_t *c, limb_t *r, const limb_t *a, const limb_t *b, const limb_t *n)
{
    oracle_bn_mul(c->prod, a, c->k, b, c->k);
    bn_mod_knuth(r, c->prod, 2 * c->k, n, c->k, c->uwork, c->vwork);
}

/* ---- exponentiation ----------------------------------------------------- */

/* Left-to-right binary method: out = base^x mod n.  base, n, out have k limbs,
 * x has xk limbs.  Returns -1 if n == 0. */
static int modexp_ltr(ctx_t *c, limb_t *out, const limb_t *base, const limb_t *x, int xk,
                      const limb_t *n, limb_t *g, limb_t *a)
{
    int k = c->k;
    int nl = bn_len(n, k);
    if (nl == 0) return -1;
    /* g = base mod n */
    bn_mod_knuth(g, base, k, n, k, c->uwork, c->vwork);
    /* A = 1 mod n */
    for (int i = 0; i < k; ++i) a[i] = 0;
    if (!(nl == 1 && n[0] == 1)) a[0] = 1;
    int xl = bn_len(x, xk);
    int top = xl ? (xl - 1) * 32 + (31 - __builtin_clz(x[xl - 1])) : -1;
    for (int bit = top; bit >= 0; --bit) {           /* t = index of the top set bit */
        modmul(c, a, a, a, n);
        if ((x[bit / 32] >> (bit % 32)) & 1u) modmul(c, a, a, g, n);
    }
    memcpy(out, a, sizeof(limb_t) * (size_t)k);
    return 0;
}

/* ---- exported single-element entry points (for the tests) -------------- */

/* r[0 .. vn-1] = u mod v by Algorithm D. */
int oracle_bn_mod(limb_t *r, const limb_t *u, int un, const limb_t *v, int vn)
{
    if (bn_len(v, vn) == 0) return -1;
    limb_t *uw = (limb_t *)malloc(sizeof(limb_t) * (size_t)(un + 2));
    limb_t *vw = (limb_t *)malloc(sizeof(limb_t) * (size_t)(vn + 1));
    if (!uw || !vw) { free(uw); free(vw); return -2; }
    bn_mod_knuth(r, u, un, v, vn, uw, vw);
    free(uw); free(vw);
    return 0;
}

/* r[0 .. vn-1] = u mod v by bit-serial shift-and-subtract. */
int oracle_bn_mod_slow(limb_t *r, const limb_t *u, int un, const limb_t *v, int vn)
{
    if (bn_len(v, vn) == 0) return -1;
    limb_t *tmp = (limb_t *)malloc(sizeof(limb_t) * (size_t)(vn + 1));
    if (!tmp) return -2;
    bn_mod_shift_subtract(r, u, un, v, vn, tmp);
    free(tmp);
    return 0;
}

/* out = base^x mod n, left-to-right binary (Fig. 5). */
int oracle_modexp(limb_t *out, const limb_t *base, const limb_t *x, const limb_t *n, int k)
{
    ctx_t c;
    if (ctx_init(&c, k)) return -2;
    limb_t *g = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    limb_t *a = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    int st = (g && a) ? modexp_ltr(&c, out, base, x, k, n, g, a) : -2;
    free(g); free(a); ctx_free(&c);
    return st;
}

/* out = base^x mod n, right-to-left binary (Fig. 5, first algorithm). */
int oracle_modexp_rtl(limb_t *out, const limb_t *base, const limb_t *x, const limb_t *n, int k)
{
    if (bn_len(n, k) == 0) return -1;
    ctx_t c;
    if (ctx_init(&c, k)) return -2;
    limb_t *s = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    limb_t *a = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    limb_t *e = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    if (!s || !a || !e) { free(s); free(a); free(e); ctx_free(&c); return -2; }
    bn_mod_knuth(s, base, k, n, k, c.uwork, c.vwork);         /* S = g mod n */
    memset(a, 0, sizeof(limb_t) * (size_t)k);                   /* A = 1 mod n */
    if (!(bn_len(n, k) == 1 && n[0] == 1)) a[0] = 1;
    memcpy(e, x, sizeof(limb_t) * (size_t)k);                   /* E = x */
    while (bn_len(e, k) != 0) {
        if (e[0] & 1u) {                 /* E odd: A = A*S, E = E - 1 */
            modmul(&c, a, a, s, n);
            e[0] &= ~1u;
        }
        for (int i = 0; i < k; ++i)      /* E = E / 2 */
            e[i] = (e[i] >> 1) | (i + 1 < k ? e[i + 1] << 31 : 0);
        if (bn_len(e, k) != 0) modmul(&c, s, s, s, n);          /* S = S*S */
    }
    memcpy(out, a, sizeof(limb_t) * (size_t)k);
    free(s); free(a); free(e); ctx_free(&c);
    return 0;
}

/* out = g^e mod n by e-1 repeated modular multiplications (Section 3.6.2,
 * Fig. 4).  e is a machine word: this is only for tiny cases.  trace, when
 * not NULL, receives the k-limb intermediate after each step (e entries). */
int oracle_modexp_naive(limb_t *out, const limb_t *g, uint64_t e, const limb_t *n, int k,
                        limb_t *trace)
{
    if (bn_len(n, k) == 0) return -1;
    ctx_t c;
    if (ctx_init(&c, k)) return -2;
    limb_t *gm = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    limb_t *acc = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    if (!gm || !acc) { free(gm); free(acc); ctx_free(&c); return -2; }
    bn_mod_knuth(gm, g, k, n, k, c.uwork, c.vwork);
    if (e == 0) {
        memset(acc, 0, sizeof(limb_t) * (size_t)k);
        if (!(bn_len(n, k) == 1 && n[0] == 1)) acc[0] = 1;
    } else {
        memcpy(acc, gm, sizeof(limb_t) * (size_t)k);            /* step 1: g mod n */
        if (trace) memcpy(trace, acc, sizeof(limb_t) * (size_t)k);
        for (uint64_t step = 2; step <= e; ++step) {
            modmul(&c, acc, acc, gm, n);
            if (trace) memcpy(trace + (size_t)(step - 1) * k, acc, sizeof(limb_t) * (size_t)k);
        }
    }
    memcpy(out, acc, sizeof(limb_t) * (size_t)k);
    free(gm); free(acc); ctx_free(&c);
    return 0;
}

/* ---- batch driver -------------------------------------------------------- */

typedef struct {
    const limb_t *base, *exp, *mod;
    limb_t *out;
    size_t begin, end;
    size_t exp_stride, mod_stride;   /* in limbs; 0 = one shared value */
    int k;
    int status;
} job_t;

static void *run_job(void *arg)
{
    job_t *j = (job_t *)arg;
    int k = j->k;
    ctx_t c;
    limb_t *g = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    limb_t *a = (limb_t *)malloc(sizeof(limb_t) * (size_t)k);
    if (ctx_init(&c, k) || !g || !a) { j->status = -2; free(g); free(a); return NULL; }
    j->status = 0;
    for (size_t i = j->begin; i < j->end; ++i) {
        int st = modexp_ltr(&c, j->out + i * (size_t)k, j->base + i * (size_t)k,
                            j->exp + i * j->exp_stride, k, j->mod + i * j->mod_stride, g, a);
        if (st) { j->status = st; break; }
    }
    free(g); free(a); ctx_free(&c);
    return NULL;
}

/*
 * out[i] = base[i]^exp[i] mod mod[i] for i < count, every number k limbs wide,
 * message-major.  exp_stride / mod_stride are the distance in limbs between
 * consecutive exponents / moduli (k for per-element values, 0 for one value
 * shared by all).  The elements are split statically over nthreads POSIX
 * threads (nthreads <= 0 means one).  Returns 0, -1 on a zero modulus, -2 on
 * allocation failure.  *wall_s receives the elapsed wall time when not NULL.
 */
int oracle_modexp_batch(const limb_t *base, const limb_t *exp, const limb_t *mod, limb_t *out,
                        size_t count, int k, size_t exp_stride, size_t mod_stride,
                        int nthreads, double *wall_s)
{
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    if (nthreads <= 0) nthreads = 1;
    if ((size_t)nthreads > count) nthreads = count ? (int)count : 1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -2; }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].base = base; jobs[t].exp = exp; jobs[t].mod = mod; jobs[t].out = out;
        jobs[t].begin = count * (size_t)t / (size_t)nthreads;
        jobs[t].end = count * (size_t)(t + 1) / (size_t)nthreads;
        jobs[t].exp_stride = exp_stride; jobs[t].mod_stride = mod_stride;
        jobs[t].k = k;
    }
    int status = 0;
    if (nthreads == 1) {
        run_job(&jobs[0]);
        status = jobs[0].status;
    } else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) {
            pthread_join(th[t], NULL);
            if (jobs[t].status && !status) status = jobs[t].status;
        }
    }
    free(jobs); free(th);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (wall_s) *wall_s = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    return status;
}
