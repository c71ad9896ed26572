/*
 * oracle/minimalist.c -- TEST INFRASTRUCTURE (the oracle).
 *
 * A plain, sequential, exact CPU implementation of the divide-and-conquer
 * kinetic 3-d convex hull that the paper runs on the GPU (Sec. 2 "Algorithm":
 * Chan's minimalist method, recast bottom-up over a movie array; Sec. 3
 * "Implementation": arrayed point lists with integer prev/next links, the act()
 * toggle of Fig. "act_functions", the event-time call of Fig.
 * "time_calculations", the level loop of Fig. "main_loop_figure" and the block
 * offsets of Fig. "kernel_variables").  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg load this file; the GPU library shares
 * no code, header, table or helper with it.
 *
 * Readings of the paper used here (the paper is silent on each):
 *  - Input is int32 x,y,z with |coord| <= 2^29; n <= 2^26.
 *  - Ties are broken by symbolic perturbation indexed by the 0-based input
 *    index i: p~ = (x + e1*i, y + e2*i^2, z + e3*i^3), 1 >> e1 >> e2 >> e3 > 0,
 *    every e_k infinitely smaller than every power of e_(k-1).  A polynomial in
 *    the e's has the sign of its first nonzero coefficient, monomials
 *    e1^a e2^b e3^c taken in ascending (c, b, a) order.
 *  - The kinetic plane at time t holds the point at (x~, z~ - t*y~).  The
 *    orientation of three points there is N - t*D, with D the xy-orientation
 *    and N the xz-orientation, so a triple is collinear at tau = N / D, the
 *    event time of the paper's time() call.
 *  - Events are ordered by (tau, key), key = the rank triple (left, middle,
 *    right) compared lexicographically; "strictly later" uses that order.
 *  - The upper hull is the lower hull of the points with z and its
 *    perturbation negated (N -> -N).
 *  - The level loop runs ceil(log2 n) levels including the final single
 *    merge; an unpaired trailing block passes through unchanged.
 *
 * Parity pins (tests/): concrete-epsilon big-integer orientation
 * (oracle/perturb.py), O(n^4) brute force, gift-wrap, Qhull, Euler count,
 * closed-manifold and containment checks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIL (-1)
#define ORACLE_MAX_N (1LL << 26)
#define ORACLE_MAX_COORD (1LL << 29)
/* The wide entry (float-lattice and lifted inputs): |x|, |y| <= 2^30,
   |z| <= 2^42.  The largest product then formed, a coefficient of
   N_A * D_B, stays below 2^200. */
#define ORACLE_MAX_XY_WIDE (1LL << 30)
#define ORACLE_MAX_Z_WIDE (1LL << 42)

/* ------------------------------------------------------------------------ */
/* Signed 256-bit integers, two's complement, four 64-bit limbs.            */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t w[4]; } i256;

static i256 big(__int128 v) {
    i256 r;
    unsigned __int128 u = (unsigned __int128)v;
    uint64_t fill = v < 0 ? ~0ULL : 0ULL;
    r.w[0] = (uint64_t)u;
    r.w[1] = (uint64_t)(u >> 64);
    r.w[2] = fill;
    r.w[3] = fill;
    return r;
}

static int big_sign(i256 a) {
    if (a.w[3] >> 63) return -1;
    return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) ? 1 : 0;
}

static i256 big_add(i256 a, i256 b) {
    i256 r;
    unsigned __int128 c = 0;
    for (int k = 0; k < 4; ++k) {
        c += (unsigned __int128)a.w[k] + b.w[k];
        r.w[k] = (uint64_t)c;
        c >>= 64;
    }
    return r;
}

static i256 big_neg(i256 a) {
    for (int k = 0; k < 4; ++k) a.w[k] = ~a.w[k];
    return big_add(a, big(1));
}

static i256 big_sub(i256 a, i256 b) { return big_add(a, big_neg(b)); }

/* Is `a` a sign-extended 64-bit value? */
static int big_fits64(i256 a) {
    uint64_t fill = (a.w[0] >> 63) ? ~0ULL : 0ULL;
    return a.w[1] == fill && a.w[2] == fill && a.w[3] == fill;
}

static i256 big_mul(i256 a, i256 b) {
    if (big_fits64(a) && big_fits64(b))
        return big((__int128)(int64_t)a.w[0] * (__int128)(int64_t)b.w[0]);
    int neg = 0;
    if (big_sign(a) < 0) { a = big_neg(a); neg ^= 1; }
    if (big_sign(b) < 0) { b = big_neg(b); neg ^= 1; }
    uint64_t prod[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) {
        unsigned __int128 carry = 0;
        for (int j = 0; j < 4; ++j) {
            unsigned __int128 t = (unsigned __int128)a.w[i] * b.w[j] + prod[i + j] + carry;
            prod[i + j] = (uint64_t)t;
            carry = t >> 64;
        }
        prod[i + 4] = (uint64_t)carry;
    }
    /* Every product formed here is bounded far below 2^255 (|x|, |y| <= 2^30,
       |z| <= 2^42, index < 2^26); anything larger is a bug, not an input
       error. */
    if (prod[4] | prod[5] | prod[6] | prod[7] | (prod[3] >> 63)) abort();
    i256 r;
    for (int k = 0; k < 4; ++k) r.w[k] = prod[k];
    return neg ? big_neg(r) : r;
}

/* ------------------------------------------------------------------------ */
/* Polynomials in (e1, e2, e3): c[e3][e2][e1], e1 <= 2, e2 <= 1, e3 <= 1.   */
/* ------------------------------------------------------------------------ */
typedef struct { i256 c[2][2][3]; } epoly;

static void ep_zero(epoly* p) { memset(p, 0, sizeof(*p)); }

static void ep_mul(const epoly* p, const epoly* q, epoly* r) {
    ep_zero(r);
    for (int c1 = 0; c1 < 2; ++c1)
        for (int b1 = 0; b1 < 2; ++b1)
            for (int a1 = 0; a1 < 3; ++a1) {
                if (!big_sign(p->c[c1][b1][a1])) continue;
                for (int c2 = 0; c2 < 2; ++c2)
                    for (int b2 = 0; b2 < 2; ++b2)
                        for (int a2 = 0; a2 < 3; ++a2) {
                            if (!big_sign(q->c[c2][b2][a2])) continue;
                            if (c1 + c2 > 1 || b1 + b2 > 1 || a1 + a2 > 2) abort();
                            r->c[c1 + c2][b1 + b2][a1 + a2] =
                                big_add(r->c[c1 + c2][b1 + b2][a1 + a2],
                                        big_mul(p->c[c1][b1][a1], q->c[c2][b2][a2]));
                        }
            }
}

static void ep_sub(const epoly* p, const epoly* q, epoly* r) {
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 3; ++a) r->c[c][b][a] = big_sub(p->c[c][b][a], q->c[c][b][a]);
}

/* Sign of a polynomial for infinitesimal e1 >> e2 >> e3: the first nonzero
   coefficient in ascending (e3, e2, e1) exponent order. */
static int ep_sign(const epoly* p) {
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 3; ++a) {
                int s = big_sign(p->c[c][b][a]);
                if (s) return s;
            }
    return 0;
}

/* Sign of p*q - r*s, taking the product coefficients one monomial at a time
   in significance order and stopping at the first nonzero one. */
static int ep_cross_sign(const epoly* p, const epoly* q, const epoly* r, const epoly* s) {
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 3; ++a) {
                i256 acc = big(0);
                for (int c1 = 0; c1 <= c; ++c1)
                    for (int b1 = 0; b1 <= b; ++b1)
                        for (int a1 = 0; a1 <= a; ++a1) {
                            int c2 = c - c1, b2 = b - b1, a2 = a - a1;
                            if (big_sign(p->c[c1][b1][a1]) && big_sign(q->c[c2][b2][a2]))
                                acc = big_add(acc, big_mul(p->c[c1][b1][a1], q->c[c2][b2][a2]));
                            if (big_sign(r->c[c1][b1][a1]) && big_sign(s->c[c2][b2][a2]))
                                acc = big_sub(acc, big_mul(r->c[c1][b1][a1], s->c[c2][b2][a2]));
                        }
                int sg = big_sign(acc);
                if (sg) return sg;
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Points (by rank) and their perturbed coordinates.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int64_t *x, *y, *z, *id; /* by rank; id = 0-based input index */
    int zsign;               /* +1: lower run; -1: upper run (z and e3 term negated) */
    int32_t *prev, *next;    /* kinetic chain links by rank, NIL = none */
    /* per-merge accounting for the bottom-up driver */
    int32_t* stamp;
    int32_t stamp_now;
    int64_t touched;
} run_t;

/* Per-level accounting: a point counts once per level when a merge of that
   level reads its coordinates (a predicate) or changes its links (act, the
   -inf splice, the rewind). */
static void touch(run_t* R, int32_t p) {
    if (p != NIL && R->stamp && R->stamp[p] != R->stamp_now) {
        R->stamp[p] = R->stamp_now;
        R->touched++;
    }
}

/* Perturbed coordinate difference coord(q) - coord(p) along one axis. */
static void pdiff(const run_t* R, int axis, int32_t p, int32_t q, epoly* out) {
    ep_zero(out);
    i256 ip = big(R->id[p]), iq = big(R->id[q]);
    if (axis == 0) {        /* x + e1 * i */
        out->c[0][0][0] = big(R->x[q] - R->x[p]);
        out->c[0][0][1] = big_sub(iq, ip);
    } else if (axis == 1) { /* y + e2 * i^2 */
        out->c[0][0][0] = big(R->y[q] - R->y[p]);
        out->c[0][1][0] = big_sub(big_mul(iq, iq), big_mul(ip, ip));
    } else {                /* zsign * (z + e3 * i^3) */
        i256 dz = big(R->z[q] - R->z[p]);
        i256 di3 = big_sub(big_mul(big_mul(iq, iq), iq), big_mul(big_mul(ip, ip), ip));
        if (R->zsign < 0) { dz = big_neg(dz); di3 = big_neg(di3); }
        out->c[0][0][0] = dz;
        out->c[1][0][0] = di3;
    }
}

/* Orientation of (a,b,c) in the plane spanned by axis 0 and axis `ax`:
   (b-a)[0]*(c-a)[ax] - (c-a)[0]*(b-a)[ax].  ax = 1 gives D, ax = 2 gives N. */
static void orient2(const run_t* R, int ax, int32_t a, int32_t b, int32_t c, epoly* out) {
    epoly bx, cx, bq, cq, t1, t2;
    pdiff(R, 0, a, b, &bx);
    pdiff(R, 0, a, c, &cx);
    pdiff(R, ax, a, b, &bq);
    pdiff(R, ax, a, c, &cq);
    ep_mul(&bx, &cq, &t1);
    ep_mul(&cx, &bq, &t2);
    ep_sub(&t1, &t2, out);
}

static int D_sign(run_t* R, int32_t a, int32_t b, int32_t c) {
    epoly d;
    touch(R, a); touch(R, b); touch(R, c);
    orient2(R, 1, a, b, c, &d);
    return ep_sign(&d);
}

/* ------------------------------------------------------------------------ */
/* Events: a rank triple (l, m, r), l < m < r, with its D and N polynomials. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int ok;
    int32_t l, m, r;
    epoly D, N;
    int dsign;
} event_t;

static void ev_make(run_t* R, event_t* e, int32_t l, int32_t m, int32_t r) {
    e->ok = 1;
    e->l = l; e->m = m; e->r = r;
    touch(R, l); touch(R, m); touch(R, r);
    orient2(R, 1, l, m, r, &e->D);
    orient2(R, 2, l, m, r, &e->N);
    e->dsign = ep_sign(&e->D);
}

/* Order of two events by (tau, key): tau = N / D compared through
   sign(tau_A - tau_B) = sign(N_A D_B - N_B D_A) * sign(D_A) * sign(D_B). */
static int ev_cmp(const event_t* A, const event_t* B) {
    int s = ep_cross_sign(&A->N, &B->D, &B->N, &A->D) * A->dsign * B->dsign;
    if (s) return s;
    if (A->l != B->l) return A->l < B->l ? -1 : 1;
    if (A->m != B->m) return A->m < B->m ? -1 : 1;
    if (A->r != B->r) return A->r < B->r ? -1 : 1;
    return 0;
}

/* The paper's act(): insert the point between its stored neighbours if the
   left neighbour does not point back at it, otherwise unlink it. */
static void act(run_t* R, int32_t p) {
    int32_t* prev = R->prev;
    int32_t* next = R->next;
    touch(R, p); touch(R, prev[p]); touch(R, next[p]);
    if (next[prev[p]] != p) {
        next[prev[p]] = p;
        prev[next[p]] = p;
    } else {
        next[prev[p]] = next[p];
        prev[next[p]] = prev[p];
    }
}

/* Merge the movies of blocks L = [s, m) and R = [m, e) (ranks) into `out`.
   On entry the links hold both blocks' chains at t = -inf, and every point not
   on them holds the neighbours it will be inserted between; on return the
   same holds for the merged block. */
static int64_t merge(run_t* R, int32_t m, const int32_t* Lmov, int64_t nL,
                     const int32_t* Rmov, int64_t nR, int32_t* out) {
    int32_t* prev = R->prev;
    int32_t* next = R->next;
    int32_t u = m - 1, v = m;

    /* Bridge at t = -inf: the lower common tangent of the two xy chains. */
    for (;;) {
        if (next[v] != NIL && D_sign(R, u, v, next[v]) < 0) v = next[v];
        else if (prev[u] != NIL && D_sign(R, prev[u], u, v) < 0) u = prev[u];
        else break;
    }

    int64_t i = 0, j = 0, k = 0;
    event_t T, c[6];
    int have_T = 0;
    for (;;) {
        for (int l = 0; l < 6; ++l) c[l].ok = 0;
        if (i < nL) ev_make(R, &c[0], prev[Lmov[i]], Lmov[i], next[Lmov[i]]);
        if (j < nR) ev_make(R, &c[1], prev[Rmov[j]], Rmov[j], next[Rmov[j]]);
        if (next[u] != NIL) ev_make(R, &c[2], u, next[u], v);
        if (prev[u] != NIL) ev_make(R, &c[3], prev[u], u, v);
        if (prev[v] != NIL) ev_make(R, &c[4], u, prev[v], v);
        if (next[v] != NIL) ev_make(R, &c[5], u, v, next[v]);
        int best = -1;
        for (int l = 0; l < 6; ++l) {
            if (!c[l].ok) continue;
            if (have_T && ev_cmp(&c[l], &T) <= 0) continue;
            if (best < 0 || ev_cmp(&c[l], &c[best]) < 0) best = l;
        }
        if (best < 0) break;
        T = c[best];
        have_T = 1;
        int32_t w;
        switch (best) {
        case 0: w = Lmov[i++]; if (w < u) out[k++] = w; act(R, w); break;
        case 1: w = Rmov[j++]; if (w > v) out[k++] = w; act(R, w); break;
        case 2: u = next[u]; out[k++] = u; break;
        case 3: out[k++] = u; u = prev[u]; break;
        case 4: v = prev[v]; out[k++] = v; break;
        default: out[k++] = v; v = next[v]; break;
        }
    }

    /* Go back in time, restoring the merged -inf chain and leaving every
       off-chain point pointing at the neighbours of its insertion. */
    touch(R, u); touch(R, v);
    next[u] = v;
    prev[v] = u;
    for (int64_t q = k - 1; q >= 0; --q) {
        int32_t w = out[q];
        if (w <= u || w >= v) {
            act(R, w);
            if (w == u) u = prev[u];
            else if (w == v) v = next[v];
        } else {
            touch(R, w); touch(R, u); touch(R, v);
            next[u] = w; prev[w] = u;
            prev[v] = w; next[w] = v;
            if (w < m) u = w; else v = w;
        }
    }
    return k;
}

/* ------------------------------------------------------------------------ */
/* Drivers.                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t* stats; /* per level: E_in, E_out, touched, merges */
    int32_t max_levels;
} stats_t;

/* Top-down recursion (Chan): the movie of ranks [s, e) goes to A + 2s, the
   children use B + 2s as their output area and A as scratch. */
static int64_t hull_topdown(run_t* R, int32_t s, int32_t e, int32_t* A, int32_t* B) {
    if (e - s == 1) {
        R->prev[s] = R->next[s] = NIL;
        return 0;
    }
    int32_t m = s + (e - s) / 2;
    int64_t nL = hull_topdown(R, s, m, B, A);
    int64_t nR = hull_topdown(R, m, e, B, A);
    return merge(R, m, B + 2 * (int64_t)s, nL, B + 2 * (int64_t)m, nR, A + 2 * (int64_t)s);
}

static int levels_for(int64_t n) {
    int L = 0;
    while ((1LL << L) < n) ++L;
    return L;
}

/* Bottom-up over the movie array (Sec. 2, Fig. "main_loop_figure" and
   "kernel_variables"): level k pairs [s, s+2^(k-1)) with [s+2^(k-1), s+2^k)
   for s = 0, 2^k, ...; the movie of block s lives at offset 2s of the level's
   output array.  Runs `upto` levels (all of them when upto < 0).  Returns the
   array holding the final movies. */
static int32_t* hull_bottomup(run_t* R, int32_t* A, int32_t* B, int64_t* lenA, int64_t* lenB,
                              int upto, stats_t* st, int64_t** len_final) {
    int64_t n = R->n;
    for (int64_t p = 0; p < n; ++p) {
        R->prev[p] = R->next[p] = NIL;
        lenA[p] = 0;
    }
    int32_t *in = A, *out = B;
    int64_t *lin = lenA, *lout = lenB;
    int L = levels_for(n);
    if (upto >= 0 && upto < L) L = upto;
    for (int k = 1; k <= L; ++k) {
        int64_t width = 1LL << k, half = width >> 1;
        int64_t e_in = 0, e_out = 0, merges = 0;
        R->touched = 0;
        R->stamp_now = k;
        for (int64_t s = 0; s < n; s += width) {
            int64_t m = s + half, e = s + width < n ? s + width : n;
            if (m >= e) { /* unpaired trailing block: passes through */
                memcpy(out + 2 * s, in + 2 * s, (size_t)lin[s] * sizeof(int32_t));
                lout[s] = lin[s];
                continue;
            }
            e_in += lin[s] + lin[m];
            lout[s] = merge(R, (int32_t)m, in + 2 * s, lin[s], in + 2 * m, lin[m], out + 2 * s);
            e_out += lout[s];
            merges++;
        }
        if (st && st->stats && k <= st->max_levels) {
            st->stats[4 * (k - 1) + 0] = e_in;
            st->stats[4 * (k - 1) + 1] = e_out;
            st->stats[4 * (k - 1) + 2] = R->touched;
            st->stats[4 * (k - 1) + 3] = merges;
        }
        int32_t* t = in; in = out; out = t;
        int64_t* tl = lin; lin = lout; lout = tl;
    }
    *len_final = lin;
    return in;
}

/* ------------------------------------------------------------------------ */
/* Setup: rank order by (x, input index).                                   */
/* ------------------------------------------------------------------------ */
static const int64_t* g_sort_xyz;
static int cmp_rank(const void* pa, const void* pb) {
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    int64_t xa = g_sort_xyz[3 * (int64_t)a], xb = g_sort_xyz[3 * (int64_t)b];
    if (xa != xb) return xa < xb ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int check_input(const int32_t* xyz, int64_t n) {
    if (n < 0 || n > ORACLE_MAX_N || (n > 0 && !xyz)) return -1;
    for (int64_t k = 0; k < 3 * n; ++k)
        if (xyz[k] > ORACLE_MAX_COORD || xyz[k] < -ORACLE_MAX_COORD) return -3;
    return 0;
}

static int check_input_wide(const int64_t* xyz, int64_t n) {
    if (n < 0 || n > ORACLE_MAX_N || (n > 0 && !xyz)) return -1;
    for (int64_t k = 0; k < n; ++k) {
        if (xyz[3 * k] > ORACLE_MAX_XY_WIDE || xyz[3 * k] < -ORACLE_MAX_XY_WIDE ||
            xyz[3 * k + 1] > ORACLE_MAX_XY_WIDE || xyz[3 * k + 1] < -ORACLE_MAX_XY_WIDE ||
            xyz[3 * k + 2] > ORACLE_MAX_Z_WIDE || xyz[3 * k + 2] < -ORACLE_MAX_Z_WIDE)
            return -3;
    }
    return 0;
}

typedef struct {
    run_t R;
    int32_t* order; /* rank -> input index */
    int32_t *A, *B;
    int64_t *lenA, *lenB;
} ctx_t;

static int ctx_init(ctx_t* C, const int64_t* xyz, int64_t n) {
    memset(C, 0, sizeof(*C));
    int64_t nn = n > 0 ? n : 1;
    C->order = malloc(sizeof(int32_t) * nn);
    C->R.x = malloc(sizeof(int64_t) * nn);
    C->R.y = malloc(sizeof(int64_t) * nn);
    C->R.z = malloc(sizeof(int64_t) * nn);
    C->R.id = malloc(sizeof(int64_t) * nn);
    C->R.prev = malloc(sizeof(int32_t) * nn);
    C->R.next = malloc(sizeof(int32_t) * nn);
    C->R.stamp = malloc(sizeof(int32_t) * nn);
    C->A = malloc(sizeof(int32_t) * 2 * nn);
    C->B = malloc(sizeof(int32_t) * 2 * nn);
    C->lenA = malloc(sizeof(int64_t) * nn);
    C->lenB = malloc(sizeof(int64_t) * nn);
    if (!C->order || !C->R.x || !C->R.y || !C->R.z || !C->R.id || !C->R.prev || !C->R.next ||
        !C->R.stamp || !C->A || !C->B || !C->lenA || !C->lenB)
        return -4;
    for (int64_t k = 0; k < n; ++k) C->order[k] = (int32_t)k;
    g_sort_xyz = xyz;
    qsort(C->order, (size_t)n, sizeof(int32_t), cmp_rank);
    for (int64_t r = 0; r < n; ++r) {
        int64_t i = C->order[r];
        C->R.x[r] = xyz[3 * i];
        C->R.y[r] = xyz[3 * i + 1];
        C->R.z[r] = xyz[3 * i + 2];
        C->R.id[r] = i;
        C->R.stamp[r] = 0;
    }
    C->R.n = n;
    return 0;
}

static void ctx_free(ctx_t* C) {
    free(C->order); free(C->R.x); free(C->R.y); free(C->R.z); free(C->R.id);
    free(C->R.prev); free(C->R.next); free(C->R.stamp);
    free(C->A); free(C->B); free(C->lenA); free(C->lenB);
}

/* ctx_init on int32 rows (widened to int64 first). */
static int ctx_init32(ctx_t* C, const int32_t* xyz, int64_t n) {
    int64_t* w = malloc(sizeof(int64_t) * 3 * (n > 0 ? n : 1));
    if (!w) { memset(C, 0, sizeof(*C)); return -4; }
    for (int64_t k = 0; k < 3 * n; ++k) w[k] = xyz[k];
    int rc = ctx_init(C, w, n);
    free(w);
    return rc;
}

/* Replay one block's movie from its -inf state: for each event w emit its
   face (prev(w), w, next(w)) and whether it is an insertion, then act(w).
   The links are restored afterwards by undoing the events in reverse. */
static void replay(run_t* R, const int32_t* mov, int64_t len, int32_t* ev4) {
    for (int64_t q = 0; q < len; ++q) {
        int32_t w = mov[q];
        ev4[4 * q + 0] = R->prev[w];
        ev4[4 * q + 1] = w;
        ev4[4 * q + 2] = R->next[w];
        ev4[4 * q + 3] = R->next[R->prev[w]] != w; /* 1 = insertion */
        act(R, w);
    }
    for (int64_t q = len - 1; q >= 0; --q) act(R, mov[q]);
}

/* ------------------------------------------------------------------------ */
/* C ABI used by the tests (ctypes).                                         */
/* ------------------------------------------------------------------------ */

/* Rank order: out[r] = input index of the point of rank r. */
int32_t oracle_sort(const int32_t* xyz, int64_t n, int32_t* out) {
    int rc = check_input(xyz, n);
    if (rc) return rc;
    ctx_t C;
    if (ctx_init32(&C, xyz, n)) { ctx_free(&C); return -4; }
    memcpy(out, C.order, sizeof(int32_t) * (size_t)n);
    ctx_free(&C);
    return 0;
}

static int32_t hull_of_ctx(ctx_t* C, int64_t n, int32_t flags, int32_t* faces,
                           int64_t* nfaces, int64_t* level_stats, int32_t max_levels) {
    int64_t F = 0;
    for (int run = 0; run < 2; ++run) {
        if (run == 0 && (flags & 4)) continue;
        if (run == 1 && (flags & 1)) continue;
        C->R.zsign = run == 0 ? 1 : -1;
        int32_t* mov;
        int64_t len;
        if (flags & 2) {
            len = hull_topdown(&C->R, 0, (int32_t)n, C->A, C->B);
            mov = C->A;
        } else {
            stats_t st = {level_stats ? level_stats + (int64_t)4 * max_levels * run : NULL, max_levels};
            int64_t* lf;
            for (int64_t p = 0; p < n; ++p) C->R.stamp[p] = 0;
            mov = hull_bottomup(&C->R, C->A, C->B, C->lenA, C->lenB, -1, &st, &lf);
            len = lf[0];
        }
        /* Output: replay from -inf, orient each face outward. */
        for (int64_t q = 0; q < len; ++q) {
            int32_t w = mov[q], a = C->R.prev[w], b = C->R.next[w];
            int ds = D_sign(&C->R, a, w, b);
            int keep = run == 0 ? ds < 0 : ds > 0; /* lower: normal z < 0 */
            int32_t p0 = a, p1 = keep ? w : b, p2 = keep ? b : w;
            faces[3 * F + 0] = C->order[p0];
            faces[3 * F + 1] = C->order[p1];
            faces[3 * F + 2] = C->order[p2];
            F++;
            act(&C->R, w);
        }
    }
    *nfaces = F;
    return 0;
}

/* Hull faces as outward (counter-clockwise seen from outside) triples of input
   indices: the lower run's faces first, then the upper run's.
   flags: 1 = lower run only, 2 = top-down driver (default bottom-up),
          4 = upper run only.
   level_stats (optional, bottom-up only): 4 int64 per level for the lower
   run then 4 per level for the upper run (E_in, E_out, touched, merges). */
int32_t oracle_hull(const int32_t* xyz, int64_t n, int32_t flags, int32_t* faces, int64_t cap,
                    int64_t* nfaces, int64_t* level_stats, int32_t max_levels) {
    int rc = check_input(xyz, n);
    if (rc) return rc;
    if (!faces || !nfaces || cap < 2 * n) return -1;
    *nfaces = 0;
    if (n < 3) return 0;
    ctx_t C;
    if (ctx_init32(&C, xyz, n)) { ctx_free(&C); return -4; }
    hull_of_ctx(&C, n, flags, faces, nfaces, level_stats, max_levels);
    ctx_free(&C);
    return 0;
}

/* oracle_hull on int64 rows over the wider range |x|, |y| <= 2^30,
   |z| <= 2^42 (lattice points of float inputs, lifted planar points); the
   same method and predicates, the same perturbation by input index. */
int32_t oracle_hull_wide(const int64_t* xyz, int64_t n, int32_t flags, int32_t* faces,
                         int64_t cap, int64_t* nfaces) {
    int rc = check_input_wide(xyz, n);
    if (rc) return rc;
    if (!faces || !nfaces || cap < 2 * n) return -1;
    *nfaces = 0;
    if (n < 3) return 0;
    ctx_t C;
    if (ctx_init(&C, xyz, n)) { ctx_free(&C); return -4; }
    hull_of_ctx(&C, n, flags, faces, nfaces, NULL, 0);
    ctx_free(&C);
    return 0;
}

/* Movies after `level` bottom-up levels (level < 0: all levels) of one run
   (0 lower, 1 upper).  For every block in rank order, its events as
   (left, middle, right, is_insertion) in ranks; block_len[b] gets the event
   count of block b (blocks of width 2^level from rank 0). */
int32_t oracle_level_movies(const int32_t* xyz, int64_t n, int32_t run, int32_t level,
                            int32_t* ev4, int64_t cap, int64_t* block_len, int64_t* total) {
    int rc = check_input(xyz, n);
    if (rc) return rc;
    *total = 0;
    if (n < 1) return 0;
    ctx_t C;
    if (ctx_init32(&C, xyz, n)) { ctx_free(&C); return -4; }
    C.R.zsign = run == 0 ? 1 : -1;
    int64_t* lf;
    int32_t* mov = hull_bottomup(&C.R, C.A, C.B, C.lenA, C.lenB, level, NULL, &lf);
    int L = levels_for(n);
    if (level >= 0 && level < L) L = level;
    int64_t width = 1LL << L, t = 0, b = 0;
    for (int64_t s = 0; s < n; s += width, ++b) {
        int64_t len = lf[s];
        if (t + len > cap) { ctx_free(&C); return -2; }
        replay(&C.R, mov + 2 * s, len, ev4 + 4 * t);
        block_len[b] = len;
        t += len;
    }
    *total = t;
    ctx_free(&C);
    return 0;
}

/* The -inf chain links after `level` bottom-up levels: prev/next by rank. */
int32_t oracle_level_chains(const int32_t* xyz, int64_t n, int32_t run, int32_t level,
                            int32_t* prev_out, int32_t* next_out) {
    int rc = check_input(xyz, n);
    if (rc) return rc;
    if (n < 1) return 0;
    ctx_t C;
    if (ctx_init32(&C, xyz, n)) { ctx_free(&C); return -4; }
    C.R.zsign = run == 0 ? 1 : -1;
    int64_t* lf;
    hull_bottomup(&C.R, C.A, C.B, C.lenA, C.lenB, level, NULL, &lf);
    /* Follow each block's chain from its leftmost rank; points off the chain
       get NIL so that only the chain is reported. */
    int L = levels_for(n);
    if (level >= 0 && level < L) L = level;
    int64_t width = 1LL << L;
    for (int64_t p = 0; p < n; ++p) prev_out[p] = next_out[p] = NIL;
    for (int64_t s = 0; s < n; s += width) {
        int32_t p = (int32_t)s;
        while (C.R.next[p] != NIL) {
            next_out[p] = C.R.next[p];
            prev_out[C.R.next[p]] = p;
            p = C.R.next[p];
        }
    }
    ctx_free(&C);
    return 0;
}

/* Exact predicate probes for the tests, on 4 points given directly as
   (x, y, z, index) rows:  which = 0: sign of D(p0,p1,p2);  1: sign of
   N(p0,p1,p2) (zsign +1);  2: sign(tau(p0,p1,p2) - tau(p0',p1',p2')) where
   the second triple is rows 3..5 (6 rows then);  3: same with zsign -1. */
int32_t oracle_predicate(const int64_t* rows, int32_t nrows, int32_t which) {
    run_t R;
    memset(&R, 0, sizeof(R));
    int64_t x[6], y[6], z[6], id[6];
    for (int k = 0; k < nrows && k < 6; ++k) {
        x[k] = rows[4 * k]; y[k] = rows[4 * k + 1]; z[k] = rows[4 * k + 2]; id[k] = rows[4 * k + 3];
    }
    R.x = x; R.y = y; R.z = z; R.id = id; R.n = nrows;
    R.zsign = which == 3 ? -1 : 1;
    epoly p;
    if (which == 0) { orient2(&R, 1, 0, 1, 2, &p); return ep_sign(&p); }
    if (which == 1) { orient2(&R, 2, 0, 1, 2, &p); return ep_sign(&p); }
    event_t A, B;
    ev_make(&R, &A, 0, 1, 2);
    ev_make(&R, &B, 3, 4, 5);
    return ep_cross_sign(&A.N, &B.D, &B.N, &A.D) * A.dsign * B.dsign;
}
