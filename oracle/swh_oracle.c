/*
 * swh_oracle.c -- plain CPU oracle for Smith-Waterman local alignment with
 * affine (Gotoh) gaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never links, includes or calls anything in this directory, and this file
 * includes nothing from the GPU library.
 *
 * Everything here is deliberately slow and direct: one cell at a time, in
 * row-major order, with 64-bit integer arithmetic so that no overflow or
 * saturation question can arise.
 *
 * What is computed (paper: Background, "Smith-Waterman algorithm (SW)" and the
 * SW# suite paragraph, which fixes the affine open/extension penalties and the
 * two phases "resolution" (maximum score) and "reconstruction" (optimal path)):
 *
 *   gap of length k costs  g(k) = o + (k-1)*e          (o > 0, 0 < e <= o)
 *   E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)           target residue vs gap  'D'
 *   F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)           query residue vs gap   'I'
 *   H(i,j) = max(0, H(i-1,j-1) + s(a_i,b_j), E(i,j), F(i,j))
 *   H(i,0) = H(0,j) = 0,  E(i,0) = F(0,j) = -inf
 *
 * Readings taken where the paper is silent (each one is listed in the design
 * notes of the repository):
 *   end   = first cell in row-major order (smallest i, then smallest j) with
 *           H = S, S = max H.  S = 0 means "no alignment".
 *   start = first cell in row-major order of the same DP run on the reversed
 *           prefixes a[1..i_end], b[1..j_end] whose value equals S.
 *   path  = greedy backward walk of the global Gotoh DP over the rectangle
 *           a[start..end] x b[start..end]: at an H node prefer the diagonal,
 *           then F ('I'), then E ('D'); inside a gap prefer closing the run
 *           (the H predecessor paying o) over extending it.
 *   CIGAR = run-length string of M / I / D, in forward order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <sched.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_ALPHABET (-2)
#define ORC_E_NOMEM (-3)
#define ORC_E_RANGE (-4)

/* Far below any reachable value; sums of a few of these cannot overflow. */
#define NEG_INF (INT64_MIN / 8)

typedef struct {
    int map[256];          /* byte -> code, -1 when not in the alphabet */
    int asize;
    const int8_t *mat;     /* asize x asize, row = query symbol */
    int64_t o, e;
} scoring;

static int64_t max2(int64_t x, int64_t y) { return x > y ? x : y; }

static int make_scoring(scoring *sc, const char *alphabet, int asize,
                        const int8_t *matrix, int o, int e)
{
    if (!alphabet || !matrix || asize <= 0 || asize > 32) return ORC_E_INVAL;
    if (o <= 0 || e <= 0 || e > o) return ORC_E_INVAL;
    for (int c = 0; c < 256; ++c) sc->map[c] = -1;
    for (int k = 0; k < asize; ++k) {
        unsigned char up = (unsigned char)alphabet[k];
        if (up >= 'a' && up <= 'z') up = (unsigned char)(up - 'a' + 'A');
        sc->map[up] = k;
        if (up >= 'A' && up <= 'Z') sc->map[up - 'A' + 'a'] = k;
    }
    sc->asize = asize;
    sc->mat = matrix;
    sc->o = o;
    sc->e = e;
    return ORC_OK;
}

/* ASCII -> codes; returns ORC_OK or ORC_E_ALPHABET with *bad = position. */
static int encode(const scoring *sc, const char *s, int64_t len, uint8_t *out, int64_t *bad)
{
    for (int64_t i = 0; i < len; ++i) {
        int c = sc->map[(unsigned char)s[i]];
        if (c < 0) { if (bad) *bad = i; return ORC_E_ALPHABET; }
        out[i] = (uint8_t)c;
    }
    return ORC_OK;
}

static int64_t subst(const scoring *sc, uint8_t x, uint8_t y)
{
    return sc->mat[(int)x * sc->asize + (int)y];
}

/*
 * Resolution phase: the local DP over a[1..n] x b[1..m], row by row.
 * Returns S and the first cell (row-major) holding S; 1-based, (0,0) if S == 0.
 */
static int local_best(const scoring *sc, const uint8_t *a, int64_t n,
                      const uint8_t *b, int64_t m,
                      int64_t *S, int64_t *ibest, int64_t *jbest)
{
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));  /* H(i-1, j) then H(i, j) */
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));  /* F(i-1, j) then F(i, j) */
    if (!H || !F) { free(H); free(F); return ORC_E_NOMEM; }
    for (int64_t j = 0; j <= m; ++j) { H[j] = 0; F[j] = NEG_INF; }
    int64_t best = 0, bi = 0, bj = 0;
    for (int64_t i = 1; i <= n; ++i) {
        int64_t diag = H[0];      /* H(i-1, 0) = 0 */
        int64_t E = NEG_INF;      /* E(i, 0) */
        H[0] = 0;                 /* H(i, 0) */
        for (int64_t j = 1; j <= m; ++j) {
            int64_t Eij = max2(E - sc->e, H[j - 1] - sc->o);      /* H[j-1] is H(i, j-1) */
            int64_t Fij = max2(F[j] - sc->e, H[j] - sc->o);       /* H[j] is H(i-1, j)   */
            int64_t h = max2(max2(0, diag + subst(sc, a[i - 1], b[j - 1])), max2(Eij, Fij));
            diag = H[j];
            H[j] = h;
            F[j] = Fij;
            E = Eij;
            if (h > best) { best = h; bi = i; bj = j; }   /* strict: keeps the first in row-major order */
        }
    }
    free(H);
    free(F);
    *S = best;
    *ibest = bi;
    *jbest = bj;
    return ORC_OK;
}

/*
 * Reconstruction phase, written as the full-matrix definition: the global
 * Gotoh DP over the rectangle A[1..p] x B[1..q] (no zero clamp), one byte of
 * tie flags per cell, then the greedy backward walk from (p, q) in state H.
 *
 * Boundary:  G(0,0) = 0;  E(i,0) = F(0,j) = -inf;  no diagonal into row 0 or
 * column 0, so G(0,j) = E(0,j) and G(i,0) = F(i,0) follow from the same
 * recurrences (a leading gap run).
 *
 * Tie flags per cell (i,j):
 *   bit 0  G == G(i-1,j-1) + s     (diagonal optimal)
 *   bit 1  G == F(i,j)
 *   bit 2  F == G(i-1,j) - o       (vertical run may be closed here)
 *   bit 3  E == G(i,j-1) - o       (horizontal run may be closed here)
 *
 * ops[] receives the op string in BACKWARD order; returns its length and the
 * final global score through *gscore.
 */
static int64_t global_walk(const scoring *sc, const uint8_t *A, int64_t p,
                           const uint8_t *B, int64_t q, char *ops, int64_t *gscore)
{
    const int64_t W = q + 1;
    uint8_t *flag = (uint8_t *)malloc((size_t)((p + 1) * W));
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);   /* row i-1, then row i */
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    if (!flag || !G || !F) { free(flag); free(G); free(F); return ORC_E_NOMEM; }

    /* row 0 */
    G[0] = 0; F[0] = NEG_INF; flag[0] = 0;
    {
        int64_t E = NEG_INF;
        for (int64_t j = 1; j <= q; ++j) {
            int64_t Ej = max2(E - sc->e, G[j - 1] - sc->o);
            uint8_t f = 0;
            if (Ej == G[j - 1] - sc->o) f |= 8;
            G[j] = Ej;           /* no diagonal, F(0,j) = -inf */
            F[j] = NEG_INF;
            E = Ej;
            flag[j] = f;
        }
    }
    for (int64_t i = 1; i <= p; ++i) {
        int64_t diag = G[0];
        int64_t E = NEG_INF;
        /* column 0: only a vertical run from the origin */
        {
            int64_t F0 = max2(F[0] - sc->e, G[0] - sc->o);
            uint8_t f = 2;                                   /* G == F */
            if (F0 == G[0] - sc->o) f |= 4;
            F[0] = F0;
            G[0] = F0;
            flag[i * W] = f;
        }
        for (int64_t j = 1; j <= q; ++j) {
            int64_t Ej = max2(E - sc->e, G[j - 1] - sc->o);
            int64_t Fj = max2(F[j] - sc->e, G[j] - sc->o);
            int64_t dj = diag + subst(sc, A[i - 1], B[j - 1]);
            int64_t g = max2(dj, max2(Ej, Fj));
            uint8_t f = 0;
            if (g == dj) f |= 1;
            if (g == Fj) f |= 2;
            if (Fj == G[j] - sc->o) f |= 4;
            if (Ej == G[j - 1] - sc->o) f |= 8;
            diag = G[j];
            G[j] = g;
            F[j] = Fj;
            E = Ej;
            flag[i * W + j] = f;
        }
    }
    *gscore = G[q];

    /* greedy backward walk */
    int64_t i = p, j = q, len = 0;
    int state = 0;   /* 0 = G, 1 = F (vertical run), 2 = E (horizontal run) */
    while (i > 0 || j > 0) {
        uint8_t f = flag[i * W + j];
        if (state == 0) {
            if (i > 0 && j > 0 && (f & 1)) { ops[len++] = 'M'; --i; --j; continue; }
            state = (f & 2) ? 1 : 2;
        } else if (state == 1) {
            ops[len++] = 'I';
            if (f & 4) state = 0;
            --i;
        } else {
            ops[len++] = 'D';
            if (f & 8) state = 0;
            --j;
        }
    }
    free(flag);
    free(G);
    free(F);
    return len;
}

/* Run-length encode ops given in backward order; returns required length. */
static int64_t cigar_from_backward(const char *ops, int64_t nops, char *out, int64_t cap)
{
    int64_t need = 0;
    char buf[32];
    int64_t k = nops - 1;
    while (k >= 0) {
        char op = ops[k];
        int64_t run = 0;
        while (k >= 0 && ops[k] == op) { ++run; --k; }
        /* format run then op */
        int d = 0;
        char tmp[24];
        int64_t r = run;
        do { tmp[d++] = (char)('0' + (r % 10)); r /= 10; } while (r);
        int w = 0;
        while (d) buf[w++] = tmp[--d];
        buf[w++] = op;
        if (out && need + w < cap) memcpy(out + need, buf, (size_t)w);
        need += w;
    }
    if (out && cap > 0) out[need < cap ? need : cap - 1] = '\0';
    return need;
}

/*
 * Full local alignment: score, 0-based inclusive coordinates and (optionally)
 * the canonical CIGAR.  coords = {q_begin, q_end, t_begin, t_end}, all -1 when
 * the score is 0.  max_cells bounds the rectangle of the full-matrix walk.
 */
int orc_sw_align(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                 const char *a, int64_t n, const char *b, int64_t m,
                 int want_cigar, int64_t max_cells,
                 int64_t *score, int64_t *coords, char *cigar, int64_t cigar_cap,
                 int64_t *cigar_len)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    if (n < 0 || m < 0 || (!a && n) || (!b && m) || !score || !coords) return ORC_E_INVAL;
    uint8_t *ca = (uint8_t *)malloc((size_t)(n + 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(m + 1));
    if (!ca || !cb) { free(ca); free(cb); return ORC_E_NOMEM; }
    int64_t bad;
    if ((rc = encode(&sc, a, n, ca, &bad)) || (rc = encode(&sc, b, m, cb, &bad))) {
        free(ca); free(cb); return rc;
    }

    int64_t S, ie, je;
    rc = local_best(&sc, ca, n, cb, m, &S, &ie, &je);
    if (rc) { free(ca); free(cb); return rc; }
    *score = S;
    coords[0] = coords[1] = coords[2] = coords[3] = -1;
    if (cigar_len) *cigar_len = 0;
    if (cigar && cigar_cap > 0) cigar[0] = '\0';
    if (S == 0) { free(ca); free(cb); return ORC_OK; }

    /* reverse pass over the prefixes that end at (ie, je) */
    uint8_t *ra = (uint8_t *)malloc((size_t)ie);
    uint8_t *rb = (uint8_t *)malloc((size_t)je);
    if (!ra || !rb) { free(ca); free(cb); free(ra); free(rb); return ORC_E_NOMEM; }
    for (int64_t k = 0; k < ie; ++k) ra[k] = ca[ie - 1 - k];
    for (int64_t k = 0; k < je; ++k) rb[k] = cb[je - 1 - k];
    int64_t S2, ri, rj;
    rc = local_best(&sc, ra, ie, rb, je, &S2, &ri, &rj);
    free(ra); free(rb);
    if (rc) { free(ca); free(cb); return rc; }
    if (S2 != S) { free(ca); free(cb); return ORC_E_INVAL; }   /* cannot happen (start lemma) */
    int64_t is = ie - ri + 1, js = je - rj + 1;                  /* 1-based starts */
    coords[0] = is - 1; coords[1] = ie - 1; coords[2] = js - 1; coords[3] = je - 1;

    if (want_cigar) {
        int64_t p = ie - is + 1, q = je - js + 1;
        if ((p + 1) * (q + 1) > max_cells) { free(ca); free(cb); return ORC_E_RANGE; }
        char *ops = (char *)malloc((size_t)(p + q + 1));
        if (!ops) { free(ca); free(cb); return ORC_E_NOMEM; }
        int64_t g;
        int64_t nops = global_walk(&sc, ca + is - 1, p, cb + js - 1, q, ops, &g);
        if (nops < 0) { free(ops); free(ca); free(cb); return (int)nops; }
        if (g != S) { free(ops); free(ca); free(cb); return ORC_E_INVAL; }
        int64_t need = cigar_from_backward(ops, nops, cigar, cigar_cap);
        free(ops);
        if (cigar_len) *cigar_len = need;
        if (!cigar || need + 1 > cigar_cap) { free(ca); free(cb); return ORC_E_RANGE; }
    }
    free(ca);
    free(cb);
    return ORC_OK;
}

/*
 * The resolution-phase DP of local_best, split over threads for one long
 * pair (the same recurrences, cell for cell; only the order in which cells
 * are visited changes).  Rows are cut into bands of `band` rows, columns into
 * chunks of `chunk` columns.  Band k visits its chunks left to right; chunk c
 * of band k needs the last row of band k-1 over the chunk's columns and the
 * left neighbours of its own rows, which band k carries from chunk c-1.  The
 * last row of a band is handed to the next band through one shared row,
 * overwritten in place one chunk at a time: band k reads chunk c, computes
 * it, writes its own last row over it and publishes progress[k] = c + 1;
 * band k+1 starts chunk c only once it sees that.  Threads take bands in
 * increasing order, so every band waits only on a band already taken.
 *
 * Because a band visits its cells chunk by chunk, the first cell in
 * row-major order holding the maximum is found by comparison (value desc,
 * row asc, column asc) rather than by visiting order.
 */
typedef struct {
    int64_t v, i, j;
} cell_pick;

/* b better than a: larger value, or equal positive value earlier in row-major order */
static int pick_better(const cell_pick *b, const cell_pick *a)
{
    if (b->v != a->v) return b->v > a->v;
    if (b->v == 0) return 0;
    if (b->i != a->i) return b->i < a->i;
    return b->j < a->j;
}

typedef struct {
    const scoring *sc;
    const uint8_t *a, *b;
    int64_t n, m, band, chunk, nbands, nchunks;
    int64_t *rowH, *rowF;          /* shared hand-over row: H, F of a band's last row, columns 1..m */
    int64_t *progress;             /* per band: chunks published (atomic) */
    int64_t next_band;             /* atomic band ticket */
    cell_pick *band_best;          /* per band */
    int status;                    /* atomic: nonzero once a worker failed */
} band_job;

static void *band_worker(void *arg)
{
    band_job *jb = (band_job *)arg;
    const scoring *sc = jb->sc;
    const int64_t B = jb->band, C = jb->chunk;
    int64_t *Hl = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);     /* H(i, c0-1) of the band's rows */
    int64_t *El = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);     /* E(i, c0-1) */
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1)); /* working row over the chunk */
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    if (!Hl || !El || !H || !F) {
        __atomic_store_n(&jb->status, ORC_E_NOMEM, __ATOMIC_RELAXED);
        free(Hl); free(El); free(H); free(F);
        return NULL;
    }
    for (;;) {
        const int64_t k = __atomic_fetch_add(&jb->next_band, 1, __ATOMIC_RELAXED);
        if (k >= jb->nbands) break;
        const int64_t top = k * B + 1, bot = (k + 1) * B < jb->n ? (k + 1) * B : jb->n;   /* rows top..bot, 1-based */
        cell_pick best = {0, 0, 0};
        for (int64_t r = 0; r < B; ++r) { Hl[r] = 0; El[r] = NEG_INF; }   /* column 0 */
        int64_t corner = 0;   /* H(top-1, c0-1): 0 on column 0 */
        for (int64_t c = 0; c < jb->nchunks; ++c) {
            const int64_t c0 = c * C + 1, c1 = (c + 1) * C < jb->m ? (c + 1) * C : jb->m;   /* columns c0..c1 */
            const int64_t w = c1 - c0 + 1;
            if (k > 0) {
                while (__atomic_load_n(&jb->progress[k - 1], __ATOMIC_ACQUIRE) <= c) {
                    if (__atomic_load_n(&jb->status, __ATOMIC_RELAXED)) goto out;
                    sched_yield();
                }
            }
            /* the row above the band over columns c0-1 .. c1: H(top-1, .), F(top-1, .) */
            H[0] = corner;
            F[0] = NEG_INF;
            for (int64_t t = 0; t < w; ++t) {
                H[t + 1] = k > 0 ? jb->rowH[c0 + t] : 0;
                F[t + 1] = k > 0 ? jb->rowF[c0 + t] : NEG_INF;
            }
            corner = H[w];   /* H(top-1, c1): the next chunk's corner */
            for (int64_t i = top; i <= bot; ++i) {
                const int64_t r = i - top;
                int64_t diag = H[0];     /* H(i-1, c0-1) */
                H[0] = Hl[r];            /* H(i, c0-1) */
                int64_t E = El[r];       /* E(i, c0-1) */
                for (int64_t t = 1; t <= w; ++t) {
                    const int64_t j = c0 + t - 1;
                    const int64_t Eij = max2(E - sc->e, H[t - 1] - sc->o);
                    const int64_t Fij = max2(F[t] - sc->e, H[t] - sc->o);
                    const int64_t h = max2(max2(0, diag + subst(sc, jb->a[i - 1], jb->b[j - 1])), max2(Eij, Fij));
                    diag = H[t];
                    H[t] = h;
                    F[t] = Fij;
                    E = Eij;
                    if (h >= best.v) {   /* only such cells can change the pick */
                        const cell_pick cp = {h, i, j};
                        if (pick_better(&cp, &best)) best = cp;
                    }
                }
                Hl[r] = H[w];
                El[r] = E;
            }
            /* hand the band's last row over this chunk to the next band */
            for (int64_t t = 0; t < w; ++t) {
                jb->rowH[c0 + t] = H[t + 1];
                jb->rowF[c0 + t] = F[t + 1];
            }
            __atomic_store_n(&jb->progress[k], c + 1, __ATOMIC_RELEASE);
        }
        jb->band_best[k] = best;
    }
out:
    free(Hl); free(El); free(H); free(F);
    return NULL;
}

static int local_best_bands(const scoring *sc, const uint8_t *a, int64_t n, const uint8_t *b, int64_t m,
                            int threads, int64_t band, int64_t chunk,
                            int64_t *S, int64_t *ibest, int64_t *jbest)
{
    *S = 0; *ibest = 0; *jbest = 0;
    if (n == 0 || m == 0) return ORC_OK;
    if (band < 1 || chunk < 1) return ORC_E_INVAL;
    band_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.sc = sc; jb.a = a; jb.b = b; jb.n = n; jb.m = m; jb.band = band; jb.chunk = chunk;
    jb.nbands = (n + band - 1) / band;
    jb.nchunks = (m + chunk - 1) / chunk;
    jb.rowH = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    jb.rowF = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    jb.progress = (int64_t *)calloc((size_t)jb.nbands, sizeof(int64_t));
    jb.band_best = (cell_pick *)calloc((size_t)jb.nbands, sizeof(cell_pick));
    if (!jb.rowH || !jb.rowF || !jb.progress || !jb.band_best) {
        free(jb.rowH); free(jb.rowF); free(jb.progress); free(jb.band_best);
        return ORC_E_NOMEM;
    }
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], NULL, band_worker, &jb) == 0) ++started;
    if (started == 0) band_worker(&jb);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    int rc = jb.status;
    if (!rc) {
        cell_pick best = {0, 0, 0};
        for (int64_t k = 0; k < jb.nbands; ++k)
            if (pick_better(&jb.band_best[k], &best)) best = jb.band_best[k];
        *S = best.v; *ibest = best.i; *jbest = best.j;
    }
    free(jb.rowH); free(jb.rowF); free(jb.progress); free(jb.band_best);
    return rc;
}

/*
 * Score, end and start of one long pair through the banded threaded pass:
 * coords = {q_begin, q_end, t_begin, t_end} (0-based, -1 when S == 0), as
 * orc_sw_align without the CIGAR.  threads, band and chunk change the
 * running time only.
 */
int orc_sw_coords_mt(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                     const char *a, int64_t n, const char *b, int64_t m,
                     int threads, int64_t band, int64_t chunk, int64_t *score, int64_t *coords)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    if (n < 0 || m < 0 || (!a && n) || (!b && m) || !score || !coords) return ORC_E_INVAL;
    uint8_t *ca = (uint8_t *)malloc((size_t)(n + 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(m + 1));
    if (!ca || !cb) { free(ca); free(cb); return ORC_E_NOMEM; }
    int64_t bad;
    if ((rc = encode(&sc, a, n, ca, &bad)) || (rc = encode(&sc, b, m, cb, &bad))) {
        free(ca); free(cb); return rc;
    }
    int64_t S, ie, je;
    rc = local_best_bands(&sc, ca, n, cb, m, threads, band, chunk, &S, &ie, &je);
    *score = S;
    coords[0] = coords[1] = coords[2] = coords[3] = -1;
    if (rc || S == 0) { free(ca); free(cb); return rc; }
    uint8_t *ra = (uint8_t *)malloc((size_t)ie);
    uint8_t *rb = (uint8_t *)malloc((size_t)je);
    if (!ra || !rb) { free(ca); free(cb); free(ra); free(rb); return ORC_E_NOMEM; }
    for (int64_t k = 0; k < ie; ++k) ra[k] = ca[ie - 1 - k];
    for (int64_t k = 0; k < je; ++k) rb[k] = cb[je - 1 - k];
    int64_t S2, ri, rj;
    rc = local_best_bands(&sc, ra, ie, rb, je, threads, band, chunk, &S2, &ri, &rj);
    free(ra); free(rb); free(ca); free(cb);
    if (rc) return rc;
    if (S2 != S) return ORC_E_INVAL;   /* cannot happen (start lemma) */
    coords[0] = ie - ri; coords[1] = ie - 1; coords[2] = je - rj; coords[3] = je - 1;
    return ORC_OK;
}

/* Score-only banded threaded pass: S and the 0-based end cell (-1 when S == 0). */
int orc_sw_end_mt(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                  const char *a, int64_t n, const char *b, int64_t m,
                  int threads, int64_t band, int64_t chunk,
                  int64_t *score, int64_t *q_end, int64_t *t_end)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    if (n < 0 || m < 0 || (!a && n) || (!b && m) || !score || !q_end || !t_end) return ORC_E_INVAL;
    uint8_t *ca = (uint8_t *)malloc((size_t)(n + 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(m + 1));
    if (!ca || !cb) { free(ca); free(cb); return ORC_E_NOMEM; }
    int64_t bad;
    if ((rc = encode(&sc, a, n, ca, &bad)) || (rc = encode(&sc, b, m, cb, &bad))) {
        free(ca); free(cb); return rc;
    }
    int64_t S, ie, je;
    rc = local_best_bands(&sc, ca, n, cb, m, threads, band, chunk, &S, &ie, &je);
    free(ca); free(cb);
    if (rc) return rc;
    *score = S;
    *q_end = ie - 1;
    *t_end = je - 1;
    return ORC_OK;
}

/* Score-only local pass: S and the 0-based end cell (-1 when S == 0). */
int orc_sw_end(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
               const char *a, int64_t n, const char *b, int64_t m,
               int64_t *score, int64_t *q_end, int64_t *t_end)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    uint8_t *ca = (uint8_t *)malloc((size_t)(n + 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(m + 1));
    if (!ca || !cb) { free(ca); free(cb); return ORC_E_NOMEM; }
    int64_t bad;
    if ((rc = encode(&sc, a, n, ca, &bad)) || (rc = encode(&sc, b, m, cb, &bad))) {
        free(ca); free(cb); return rc;
    }
    int64_t S, ie, je;
    rc = local_best(&sc, ca, n, cb, m, &S, &ie, &je);
    free(ca); free(cb);
    if (rc) return rc;
    *score = S;
    *q_end = ie - 1;
    *t_end = je - 1;
    return ORC_OK;
}

/*
 * Global rectangle walk exposed on its own (used by tests to check the
 * reconstruction phase on inputs chosen directly).  Returns the global
 * optimum through *gscore and the CIGAR.
 */
int orc_global_cigar(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                     const char *a, int64_t p, const char *b, int64_t q,
                     int64_t *gscore, char *cigar, int64_t cigar_cap, int64_t *cigar_len)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    uint8_t *ca = (uint8_t *)malloc((size_t)(p + 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(q + 1));
    char *ops = (char *)malloc((size_t)(p + q + 1));
    if (!ca || !cb || !ops) { free(ca); free(cb); free(ops); return ORC_E_NOMEM; }
    int64_t bad;
    if ((rc = encode(&sc, a, p, ca, &bad)) || (rc = encode(&sc, b, q, cb, &bad))) {
        free(ca); free(cb); free(ops); return rc;
    }
    int64_t nops = global_walk(&sc, ca, p, cb, q, ops, gscore);
    free(ca); free(cb);
    if (nops < 0) { free(ops); return (int)nops; }
    int64_t need = cigar_from_backward(ops, nops, cigar, cigar_cap);
    free(ops);
    if (cigar_len) *cigar_len = need;
    if (!cigar || need + 1 > cigar_cap) return ORC_E_RANGE;
    return ORC_OK;
}

/*
 * Semi-global alignment (paper, Background, "Semi-global algorithm (HW)").
 * Reading: the whole query against a part of the target whose surrounding
 * target residues are not penalised; gaps at the ends of the query are.
 *   G(0,j) = 0 (free leading target), G(i,0) = -(o + (i-1) e), E and F as
 *   for the local DP, no zero floor; S = max_j G(n, j) (free trailing
 *   target), end = the smallest such j (the first cell in row-major order).
 *   start: the same DP on the reversed query and reversed target prefix
 *   b[1..je], entered at its corner (top border -(o + (j-1) e)): its last
 *   row holds at column c the best alignment of the whole query against
 *   b[je-c+1..je]; the smallest c with value S gives the largest start.
 *   path: the greedy walk of the global DP over a x b[js..je].
 * An alignment with no target residue (S = G(n, 0)) has t_begin = t_end = -1
 * and the CIGAR "nI"; an empty query scores 0 with no alignment.
 */
static int64_t *hw_last_row(const scoring *sc, const uint8_t *A, int64_t n, const uint8_t *B, int64_t m,
                            int free_top)
{
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!G || !F) { free(G); free(F); return NULL; }
    G[0] = 0;
    F[0] = NEG_INF;
    for (int64_t j = 1; j <= m; ++j) {
        G[j] = free_top ? 0 : -(sc->o + (j - 1) * sc->e);
        F[j] = NEG_INF;
    }
    for (int64_t i = 1; i <= n; ++i) {
        int64_t diag = G[0];
        F[0] = max2(F[0] - sc->e, G[0] - sc->o);
        G[0] = F[0];
        int64_t E = NEG_INF;
        for (int64_t j = 1; j <= m; ++j) {
            int64_t Ej = max2(E - sc->e, G[j - 1] - sc->o);
            int64_t Fj = max2(F[j] - sc->e, G[j] - sc->o);
            int64_t g = max2(diag + subst(sc, A[i - 1], B[j - 1]), max2(Ej, Fj));
            diag = G[j];
            G[j] = g;
            F[j] = Fj;
            E = Ej;
        }
    }
    free(F);
    return G;
}

int orc_hw_align(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                 const char *a, int64_t n, const char *b, int64_t m, int want_cigar,
                 int64_t *score, int64_t *coords, char *cigar, int64_t cigar_cap, int64_t *cigar_len)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    if (n < 0 || m < 0 || (!a && n) || (!b && m) || !score || !coords) return ORC_E_INVAL;
    coords[0] = coords[1] = coords[2] = coords[3] = -1;
    *score = 0;
    if (cigar_len) *cigar_len = 0;
    if (cigar && cigar_cap > 0) cigar[0] = '\0';
    if (n == 0) return ORC_OK;
    uint8_t *ca = (uint8_t *)malloc((size_t)(n + 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(m + 1));
    if (!ca || !cb) { free(ca); free(cb); return ORC_E_NOMEM; }
    int64_t bad;
    if ((rc = encode(&sc, a, n, ca, &bad)) || (rc = encode(&sc, b, m, cb, &bad))) {
        free(ca); free(cb); return rc;
    }
    int64_t *row = hw_last_row(&sc, ca, n, cb, m, 1);
    if (!row) { free(ca); free(cb); return ORC_E_NOMEM; }
    int64_t S = row[0], je = 0;
    for (int64_t j = 1; j <= m; ++j)
        if (row[j] > S) { S = row[j]; je = j; }
    free(row);
    *score = S;
    coords[0] = 0;
    coords[1] = n - 1;
    int64_t js = 1;
    if (je > 0) {
        uint8_t *ra = (uint8_t *)malloc((size_t)n);
        uint8_t *rb = (uint8_t *)malloc((size_t)je);
        if (!ra || !rb) { free(ra); free(rb); free(ca); free(cb); return ORC_E_NOMEM; }
        for (int64_t k = 0; k < n; ++k) ra[k] = ca[n - 1 - k];
        for (int64_t k = 0; k < je; ++k) rb[k] = cb[je - 1 - k];
        int64_t *rrow = hw_last_row(&sc, ra, n, rb, je, 0);
        free(ra); free(rb);
        if (!rrow) { free(ca); free(cb); return ORC_E_NOMEM; }
        int64_t c = 1;
        while (c <= je && rrow[c] != S) ++c;
        free(rrow);
        if (c > je) { free(ca); free(cb); return ORC_E_INVAL; }   /* cannot happen */
        js = je - c + 1;
        coords[2] = js - 1;
        coords[3] = je - 1;
    }
    if (want_cigar) {
        const int64_t q = je > 0 ? je - js + 1 : 0;
        char *ops = (char *)malloc((size_t)(n + q + 1));
        if (!ops) { free(ca); free(cb); return ORC_E_NOMEM; }
        int64_t g;
        int64_t nops = global_walk(&sc, ca, n, cb + (je > 0 ? js - 1 : 0), q, ops, &g);
        if (nops < 0) { free(ops); free(ca); free(cb); return (int)nops; }
        if (g != S) { free(ops); free(ca); free(cb); return ORC_E_INVAL; }
        int64_t need = cigar_from_backward(ops, nops, cigar, cigar_cap);
        free(ops);
        if (cigar_len) *cigar_len = need;
        if (!cigar || need + 1 > cigar_cap) { free(ca); free(cb); return ORC_E_RANGE; }
    }
    free(ca);
    free(cb);
    return ORC_OK;
}

/*
 * Overlap alignment (paper, Background, "Overlap algorithm (OV)"): both
 * sequences aligned end to end except that gaps before the first and after
 * the last aligned residue of either sequence cost nothing.
 *   G(0,j) = G(i,0) = 0, E and F as for the local DP, no zero floor;
 *   S = the maximum over the last column G(i, m) and the last row G(n, j).
 *   end: the first cell of that border in row-major order holding S (the
 *   last column above row n, then the last row from the left).
 *   start: the DP on the reversed prefixes a[1..ie], b[1..je] entered at its
 *   corner (both borders penalised: G'(0,c) = -(o + (c-1) e), the same down
 *   the first column); its last column and last row hold the best alignments
 *   that start on the forward top row or left column and end at (ie, je);
 *   the first of them in row-major order holding S gives the largest start.
 *   path: the greedy walk of the global DP over a[is+1..ie] x b[js+1..je].
 * S = 0 (the empty overlap is always available) reports no alignment, as the
 * local form does: all coordinates -1 and an empty CIGAR.
 */
static int ov_borders(const scoring *sc, const uint8_t *A, int64_t n, const uint8_t *B, int64_t m,
                      int free_start, int64_t *last_row, int64_t *last_col)
{
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!G || !F) { free(G); free(F); return ORC_E_NOMEM; }
    G[0] = 0;
    F[0] = NEG_INF;
    for (int64_t j = 1; j <= m; ++j) {
        G[j] = free_start ? 0 : -(sc->o + (j - 1) * sc->e);
        F[j] = NEG_INF;
    }
    last_col[0] = G[m];
    for (int64_t i = 1; i <= n; ++i) {
        int64_t diag = G[0];
        if (free_start) {
            G[0] = 0;
        } else {
            F[0] = max2(F[0] - sc->e, G[0] - sc->o);
            G[0] = F[0];
        }
        int64_t E = NEG_INF;
        for (int64_t j = 1; j <= m; ++j) {
            int64_t Ej = max2(E - sc->e, G[j - 1] - sc->o);
            int64_t Fj = max2(F[j] - sc->e, G[j] - sc->o);
            int64_t g = max2(diag + subst(sc, A[i - 1], B[j - 1]), max2(Ej, Fj));
            diag = G[j];
            G[j] = g;
            F[j] = Fj;
            E = Ej;
        }
        last_col[i] = G[m];
    }
    memcpy(last_row, G, sizeof(int64_t) * (size_t)(m + 1));
    free(G);
    free(F);
    return ORC_OK;
}

/* First border cell in row-major order holding S: (row, col) of the cell. */
static int ov_pick(const int64_t *last_row, const int64_t *last_col, int64_t n, int64_t m, int64_t S,
                   int64_t *r, int64_t *c)
{
    for (int64_t i = 0; i < n; ++i)
        if (last_col[i] == S) { *r = i; *c = m; return 1; }
    for (int64_t j = 0; j <= m; ++j)
        if (last_row[j] == S) { *r = n; *c = j; return 1; }
    return 0;
}

int orc_ov_align(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                 const char *a, int64_t n, const char *b, int64_t m, int want_cigar,
                 int64_t *score, int64_t *coords, char *cigar, int64_t cigar_cap, int64_t *cigar_len)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    if (n < 0 || m < 0 || (!a && n) || (!b && m) || !score || !coords) return ORC_E_INVAL;
    coords[0] = coords[1] = coords[2] = coords[3] = -1;
    *score = 0;
    if (cigar_len) *cigar_len = 0;
    if (cigar && cigar_cap > 0) cigar[0] = '\0';
    if (n == 0 || m == 0) return ORC_OK;
    uint8_t *ca = (uint8_t *)malloc((size_t)n);
    uint8_t *cb = (uint8_t *)malloc((size_t)m);
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!ca || !cb || !row || !col) { rc = ORC_E_NOMEM; goto out; }
    int64_t bad;
    if ((rc = encode(&sc, a, n, ca, &bad)) || (rc = encode(&sc, b, m, cb, &bad))) goto out;
    if ((rc = ov_borders(&sc, ca, n, cb, m, 1, row, col))) goto out;
    int64_t S = 0;
    for (int64_t i = 0; i <= n; ++i) S = max2(S, col[i]);
    for (int64_t j = 0; j <= m; ++j) S = max2(S, row[j]);
    *score = S;
    if (S == 0) goto out;
    int64_t ie, je;
    ov_pick(row, col, n, m, S, &ie, &je);
    /* reversed prefixes: row r of the reversed DP is query residue ie - r + 1 */
    {
        uint8_t *ra = (uint8_t *)malloc((size_t)ie);
        uint8_t *rb = (uint8_t *)malloc((size_t)je);
        int64_t *rrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)(je + 1));
        int64_t *rcol = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ie + 1));
        if (!ra || !rb || !rrow || !rcol) {
            free(ra); free(rb); free(rrow); free(rcol);
            rc = ORC_E_NOMEM;
            goto out;
        }
        for (int64_t k = 0; k < ie; ++k) ra[k] = ca[ie - 1 - k];
        for (int64_t k = 0; k < je; ++k) rb[k] = cb[je - 1 - k];
        rc = ov_borders(&sc, ra, ie, rb, je, 0, rrow, rcol);
        int64_t r = -1, c = -1;
        const int found = rc == ORC_OK && ov_pick(rrow, rcol, ie, je, S, &r, &c);
        free(ra); free(rb); free(rrow); free(rcol);
        if (rc) goto out;
        if (!found) { rc = ORC_E_INVAL; goto out; }   /* cannot happen */
        const int64_t is = ie - r, js = je - c;
        coords[0] = is;
        coords[1] = ie - 1;
        coords[2] = js;
        coords[3] = je - 1;
        if (want_cigar) {
            char *ops = (char *)malloc((size_t)(ie - is + je - js + 1));
            if (!ops) { rc = ORC_E_NOMEM; goto out; }
            int64_t g;
            int64_t nops = global_walk(&sc, ca + is, ie - is, cb + js, je - js, ops, &g);
            if (nops < 0) { free(ops); rc = (int)nops; goto out; }
            if (g != S) { free(ops); rc = ORC_E_INVAL; goto out; }
            int64_t need = cigar_from_backward(ops, nops, cigar, cigar_cap);
            free(ops);
            if (cigar_len) *cigar_len = need;
            if (!cigar || need + 1 > cigar_cap) rc = ORC_E_RANGE;
        }
    }
out:
    free(ca); free(cb); free(row); free(col);
    return rc;
}

/* ---- many independent pairs / database search (threads over units) ---- */

typedef struct {
    const scoring *sc;
    const uint8_t *qc; const int64_t *qo;
    const uint8_t *dc; const int64_t *dof;
    int64_t nq, ndb;
    int64_t next;            /* shared unit counter */
    pthread_mutex_t mu;
    int64_t *scores;         /* nq * ndb */
    int status;
} db_job;

static void *db_worker(void *arg)
{
    db_job *jb = (db_job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int64_t u = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (u >= jb->nq * jb->ndb) break;
        int64_t qi = u / jb->ndb, di = u % jb->ndb;
        int64_t S, bi, bj;
        int rc = local_best(jb->sc, jb->qc + jb->qo[qi], jb->qo[qi + 1] - jb->qo[qi],
                            jb->dc + jb->dof[di], jb->dof[di + 1] - jb->dof[di], &S, &bi, &bj);
        if (rc) { jb->status = rc; break; }
        jb->scores[u] = S;
    }
    return NULL;
}

/*
 * Scores of every (query, db sequence) pair: scores[qi * ndb + di] = S.
 * Sequences are concatenated ASCII with int64 offsets (length = count + 1).
 */
int orc_db_scores(const char *alphabet, int asize, const int8_t *matrix, int o, int e,
                  int64_t nq, const char *q_cat, const int64_t *q_off,
                  int64_t ndb, const char *db_cat, const int64_t *db_off,
                  int threads, int64_t *scores)
{
    scoring sc;
    int rc = make_scoring(&sc, alphabet, asize, matrix, o, e);
    if (rc) return rc;
    if (nq < 0 || ndb < 0 || !q_off || !db_off || !scores) return ORC_E_INVAL;
    int64_t ql = q_off[nq] - q_off[0], dl = db_off[ndb] - db_off[0];
    uint8_t *qc = (uint8_t *)malloc((size_t)(ql + 1));
    uint8_t *dc = (uint8_t *)malloc((size_t)(dl + 1));
    int64_t *qo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nq + 1));
    int64_t *dofs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ndb + 1));
    if (!qc || !dc || !qo || !dofs) { free(qc); free(dc); free(qo); free(dofs); return ORC_E_NOMEM; }
    int64_t bad;
    rc = encode(&sc, q_cat + q_off[0], ql, qc, &bad);
    if (!rc) rc = encode(&sc, db_cat + db_off[0], dl, dc, &bad);
    if (rc) { free(qc); free(dc); free(qo); free(dofs); return rc; }
    for (int64_t k = 0; k <= nq; ++k) qo[k] = q_off[k] - q_off[0];
    for (int64_t k = 0; k <= ndb; ++k) dofs[k] = db_off[k] - db_off[0];

    db_job jb;
    jb.sc = &sc; jb.qc = qc; jb.qo = qo; jb.dc = dc; jb.dof = dofs;
    jb.nq = nq; jb.ndb = ndb; jb.next = 0; jb.scores = scores; jb.status = ORC_OK;
    pthread_mutex_init(&jb.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], NULL, db_worker, &jb) == 0) ++started;
    if (started == 0) db_worker(&jb);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&jb.mu);
    free(qc); free(dc); free(qo); free(dofs);
    return jb.status;
}

/* Top-k of one score row: score descending, then index ascending. */
typedef struct { int64_t score, idx; } hit;

static int hit_cmp(const void *x, const void *y)
{
    const hit *a = (const hit *)x, *b = (const hit *)y;
    if (a->score != b->score) return a->score > b->score ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

int orc_topk(int64_t nrows, int64_t ncols, const int64_t *scores, int64_t k,
             int64_t *out_idx, int64_t *out_score)
{
    if (nrows < 0 || ncols < 0 || k < 0) return ORC_E_INVAL;
    hit *h = (hit *)malloc(sizeof(hit) * (size_t)(ncols + 1));
    if (!h) return ORC_E_NOMEM;
    for (int64_t r = 0; r < nrows; ++r) {
        for (int64_t c = 0; c < ncols; ++c) { h[c].score = scores[r * ncols + c]; h[c].idx = c; }
        qsort(h, (size_t)ncols, sizeof(hit), hit_cmp);
        for (int64_t t = 0; t < k; ++t) {
            out_idx[r * k + t] = t < ncols ? h[t].idx : -1;
            out_score[r * k + t] = t < ncols ? h[t].score : -1;
        }
    }
    free(h);
    return ORC_OK;
}
