/*
 * oracle/gotoh.c -- CPU oracle for batched Smith-Waterman with affine gaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code.  It shares no code, header,
 * table or helper with the GPU library and is deliberately plain: full
 * matrices, scalar loops, no blocking, no SIMD.
 *
 * What it computes (Sec. 2, "Stage E: SWA + Splice Junctions", task iii): the
 * read is aligned against each candidate window (extended CAL) with the
 * Smith-Waterman local alignment algorithm, returning the alignment, its score
 * and its start position.  The paper leaves the scoring model open; this
 * oracle uses Gotoh's affine-gap formulation with signed integer scores
 * (match > 0, mismatch, gap_open, gap_extend), where a gap of k bases costs
 * gap_open + (k-1)*gap_extend:
 *
 *   H(i,0) = H(0,j) = 0,   E(i,0) = F(0,j) = NEG
 *   E(i,j) = max(H(i,j-1) + gap_open, E(i,j-1) + gap_extend)   deletion  (consumes window)
 *   F(i,j) = max(H(i-1,j) + gap_open, F(i-1,j) + gap_extend)   insertion (consumes read)
 *   H(i,j) = max(0, H(i-1,j-1) + s(q_i, r_j), E(i,j), F(i,j))
 *   S = max over i>=1, j>=1 of H(i,j)  (0 when either sequence is empty)
 *
 * End cell: among cells with H == S the smallest j (window position), then the
 * smallest i.  Canonical traceback from the end cell, in state H:
 *   H: stop if H == 0; else diagonal (M) if H == H(i-1,j-1)+s; else E; else F.
 *   E: emit D; go to H at (i,j-1) if E == H(i,j-1)+gap_open, else stay in E.
 *   F: emit I; go to H at (i-1,j) if F == H(i-1,j)+gap_open, else stay in F.
 * The CIGAR is the reversed op list, run-length encoded as uint32
 * (len << 4 | op) with M=0, I=1, D=2, S=4, plus soft clips for the unaligned
 * read prefix and suffix.  Coordinates are 0-based inclusive; window
 * coordinates are relative to the window start.  A pair with S == 0 reports
 * all coordinates as -1 and no ops.
 *
 * Strand: a window with strand 1 is aligned against the reverse complement of
 * the read (Sec. 2, Stage B: alignment records carry the strand).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NEG (-(1 << 30))

typedef struct {
    int32_t match, mismatch, gap_open, gap_extend;
} orc_scoring;

typedef struct {
    int32_t score, read_begin, read_end, ref_begin, ref_end;
    uint32_t n_ops, status;   /* status bit0: ops truncated, bit1: invalid pair */
} orc_result;

enum { OP_M = 0, OP_I = 1, OP_D = 2, OP_S = 4 };

static int code_of(uint8_t c)
{
    switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
    }
}

static int imax(int a, int b) { return a > b ? a : b; }

/* Full-matrix Gotoh with canonical traceback.  q, r are codes 0..3. */
static void align_full(const uint8_t *q, int m, const uint8_t *r, int n, const orc_scoring *sc,
                       int want_ops, orc_result *res, uint32_t *ops, uint32_t ops_cap)
{
    res->score = 0;
    res->read_begin = res->read_end = res->ref_begin = res->ref_end = -1;
    res->n_ops = 0;
    res->status = 0;
    if (m <= 0 || n <= 0)
        return;
    const int W = n + 1;
    int *H = malloc(sizeof(int) * (size_t)(m + 1) * W);
    int *E = malloc(sizeof(int) * (size_t)(m + 1) * W);
    int *F = malloc(sizeof(int) * (size_t)(m + 1) * W);
#define AT(X, i, j) X[(size_t)(i) * W + (j)]
    for (int j = 0; j <= n; j++) {
        AT(H, 0, j) = 0;
        AT(E, 0, j) = NEG;
        AT(F, 0, j) = NEG;
    }
    for (int i = 1; i <= m; i++) {
        AT(H, i, 0) = 0;
        AT(E, i, 0) = NEG;
        AT(F, i, 0) = NEG;
        for (int j = 1; j <= n; j++) {
            int s = (q[i - 1] == r[j - 1]) ? sc->match : sc->mismatch;
            int e = imax(AT(H, i, j - 1) + sc->gap_open, AT(E, i, j - 1) + sc->gap_extend);
            int f = imax(AT(H, i - 1, j) + sc->gap_open, AT(F, i - 1, j) + sc->gap_extend);
            int h = imax(imax(0, AT(H, i - 1, j - 1) + s), imax(e, f));
            AT(E, i, j) = e;
            AT(F, i, j) = f;
            AT(H, i, j) = h;
        }
    }
    /* S, then the end cell: smallest j, then smallest i */
    int S = 0;
    for (int i = 1; i <= m; i++)
        for (int j = 1; j <= n; j++)
            S = imax(S, AT(H, i, j));
    if (S == 0)
        goto done;
    int ei = -1, ej = -1;
    for (int j = 1; j <= n && ei < 0; j++)
        for (int i = 1; i <= m; i++)
            if (AT(H, i, j) == S) {
                ei = i;
                ej = j;
                break;
            }
    res->score = S;
    res->read_end = ei - 1;
    res->ref_end = ej - 1;

    /* canonical traceback; ops collected backwards, one per column/row step */
    uint8_t *rev = malloc((size_t)(m + n + 2));
    int nrev = 0;
    int i = ei, j = ej, state = 0; /* 0 = H, 1 = E, 2 = F */
    int bi = ei, bj = ej;
    for (;;) {
        if (state == 0) {
            int h = AT(H, i, j);
            if (h == 0)
                break;
            int s = (q[i - 1] == r[j - 1]) ? sc->match : sc->mismatch;
            if (h == AT(H, i - 1, j - 1) + s) {
                rev[nrev++] = OP_M;
                bi = i;
                bj = j;
                i--;
                j--;
            } else if (h == AT(E, i, j)) {
                state = 1;
            } else {
                state = 2;
            }
        } else if (state == 1) {
            rev[nrev++] = OP_D;
            if (AT(E, i, j) == AT(H, i, j - 1) + sc->gap_open)
                state = 0;
            j--;
        } else {
            rev[nrev++] = OP_I;
            if (AT(F, i, j) == AT(H, i - 1, j) + sc->gap_open)
                state = 0;
            i--;
        }
    }
    res->read_begin = bi - 1;
    res->ref_begin = bj - 1;

    if (want_ops) {
        uint32_t cnt = 0;
        int trunc = 0;
#define PUSH(len, op)                                                   \
    do {                                                                \
        if (cnt < ops_cap) ops[cnt] = ((uint32_t)(len) << 4) | (op);    \
        else trunc = 1;                                                 \
        cnt++;                                                          \
    } while (0)
        if (res->read_begin > 0)
            PUSH(res->read_begin, OP_S);
        int k = nrev - 1;
        while (k >= 0) {
            int op = rev[k], len = 0;
            while (k >= 0 && rev[k] == op) {
                len++;
                k--;
            }
            PUSH(len, op);
        }
        if (m - 1 - res->read_end > 0)
            PUSH(m - 1 - res->read_end, OP_S);
#undef PUSH
        res->n_ops = trunc ? ops_cap : cnt;
        if (trunc)
            res->status |= 1;
    }
    free(rev);
done:
    free(H);
    free(E);
    free(F);
#undef AT
}

/* Scores and end cell only, two rows of memory. */
static void score_linear(const uint8_t *q, int m, const uint8_t *r, int n, const orc_scoring *sc,
                         orc_result *res, int *Hrow, int *Frow)
{
    res->score = 0;
    res->read_begin = res->read_end = res->ref_begin = res->ref_end = -1;
    res->n_ops = 0;
    res->status = 0;
    if (m <= 0 || n <= 0)
        return;
    for (int j = 0; j <= n; j++) {
        Hrow[j] = 0;      /* H(i-1, j) */
        Frow[j] = NEG;    /* F(i-1, j) */
    }
    int best = 0, bi = -1, bj = -1;
    for (int i = 1; i <= m; i++) {
        int diag = 0;     /* H(i-1, j-1) */
        int hleft = 0;    /* H(i, j-1) */
        int e = NEG;      /* E(i, j-1) */
        for (int j = 1; j <= n; j++) {
            int s = (q[i - 1] == r[j - 1]) ? sc->match : sc->mismatch;
            e = imax(hleft + sc->gap_open, e + sc->gap_extend);
            int f = imax(Hrow[j] + sc->gap_open, Frow[j] + sc->gap_extend);
            int h = imax(imax(0, diag + s), imax(e, f));
            diag = Hrow[j];
            Hrow[j] = h;
            Frow[j] = f;
            hleft = h;
            if (h > best || (h == best && h > 0 && j < bj)) {
                best = h;
                bi = i;
                bj = j;
            }
        }
    }
    if (best > 0) {
        res->score = best;
        res->read_end = bi - 1;
        res->ref_end = bj - 1;
    }
}

typedef struct {
    const uint8_t *ref;
    uint64_t ref_len;
    const uint8_t *reads;
    const uint64_t *read_off;
    const uint16_t *read_len;
    uint32_t n_reads;
    const uint8_t *win;        /* 12-byte records: u32 read_id, u32 ref_begin, u16 len, u8 strand, u8 flags */
    const uint32_t *sel;       /* optional list of pair indices */
    uint32_t n_work;
    orc_scoring sc;
    int mode;                  /* 0: score + end (linear), 1: full alignment + ops */
    orc_result *out;
    uint32_t *ops;
    uint32_t ops_stride;
    volatile uint32_t next;
    pthread_mutex_t lock;
    int bad_input;
} job_t;

static void run_pair(job_t *jb, uint32_t k, uint8_t *qbuf, uint8_t *rbuf, int *Hrow, int *Frow)
{
    uint32_t p = jb->sel ? jb->sel[k] : k;
    const uint8_t *w = jb->win + (size_t)p * 12;
    uint32_t read_id, ref_begin;
    uint16_t len;
    memcpy(&read_id, w, 4);
    memcpy(&ref_begin, w + 4, 4);
    memcpy(&len, w + 8, 2);
    uint8_t strand = w[10];
    orc_result *res = &jb->out[k];
    if (read_id >= jb->n_reads) {
        res->score = -1;
        res->read_begin = res->read_end = res->ref_begin = res->ref_end = -1;
        res->n_ops = 0;
        res->status = 2;
        return;
    }
    int m = jb->read_len[read_id];
    const uint8_t *rd = jb->reads + jb->read_off[read_id];
    for (int i = 0; i < m; i++) {
        int c = strand ? code_of(rd[m - 1 - i]) : code_of(rd[i]);
        if (c < 0) {
            jb->bad_input = 1;
            c = 0;
        }
        qbuf[i] = (uint8_t)(strand ? 3 - c : c);
    }
    int n = 0;
    if ((uint64_t)ref_begin < jb->ref_len) {
        uint64_t avail = jb->ref_len - ref_begin;
        n = (int)(len < avail ? len : avail);
    }
    for (int j = 0; j < n; j++) {
        int c = code_of(jb->ref[ref_begin + j]);
        if (c < 0) {
            jb->bad_input = 1;
            c = 0;
        }
        rbuf[j] = (uint8_t)c;
    }
    if (jb->mode == 0)
        score_linear(qbuf, m, rbuf, n, &jb->sc, res, Hrow, Frow);
    else
        align_full(qbuf, m, rbuf, n, &jb->sc, 1, res,
                   jb->ops ? jb->ops + (size_t)k * jb->ops_stride : NULL,
                   jb->ops ? jb->ops_stride : 0);
}

static void *worker(void *arg)
{
    job_t *jb = arg;
    uint8_t *qbuf = malloc(65536);
    uint8_t *rbuf = malloc(65536);
    int *Hrow = malloc(sizeof(int) * 65537);
    int *Frow = malloc(sizeof(int) * 65537);
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        uint32_t k0 = jb->next;
        jb->next = k0 + 16;
        pthread_mutex_unlock(&jb->lock);
        if (k0 >= jb->n_work)
            break;
        uint32_t k1 = k0 + 16 < jb->n_work ? k0 + 16 : jb->n_work;
        for (uint32_t k = k0; k < k1; k++)
            run_pair(jb, k, qbuf, rbuf, Hrow, Frow);
    }
    free(qbuf);
    free(rbuf);
    free(Hrow);
    free(Frow);
    return NULL;
}

/*
 * Align every pair (or the pairs listed in `sel`, if not NULL) of a batch.
 * Sequences are ASCII; windows are 12-byte records.  mode 0 fills score and
 * end coordinates; mode 1 also fills begin coordinates and CIGAR ops
 * (ops_stride uint32 slots per pair).  Returns 0, or -1 on a non-ACGT base.
 */
int orc_batch(const uint8_t *ref, uint64_t ref_len, const uint8_t *reads, const uint64_t *read_off,
              const uint16_t *read_len, uint32_t n_reads, const uint8_t *win, const uint32_t *sel,
              uint32_t n_work, const orc_scoring *sc, int mode, orc_result *out, uint32_t *ops,
              uint32_t ops_stride, int nthreads)
{
    job_t jb;
    memset(&jb, 0, sizeof jb);
    jb.ref = ref;
    jb.ref_len = ref_len;
    jb.reads = reads;
    jb.read_off = read_off;
    jb.read_len = read_len;
    jb.n_reads = n_reads;
    jb.win = win;
    jb.sel = sel;
    jb.n_work = n_work;
    jb.sc = *sc;
    jb.mode = mode;
    jb.out = out;
    jb.ops = ops;
    jb.ops_stride = ops_stride;
    jb.next = 0;
    pthread_mutex_init(&jb.lock, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++)
        pthread_create(&th[t], NULL, worker, &jb);
    for (int t = 0; t < nthreads; t++)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb.lock);
    return jb.bad_input ? -1 : 0;
}

/* Single pair on codes (0..3), full alignment: used by the unit tests. */
int orc_align_codes(const uint8_t *q, int m, const uint8_t *r, int n, const orc_scoring *sc,
                    orc_result *res, uint32_t *ops, uint32_t ops_cap)
{
    align_full(q, m, r, n, sc, 1, res, ops, ops_cap);
    return 0;
}

/* Single pair on codes, linear-memory score + end: used by the unit tests. */
int orc_score_codes(const uint8_t *q, int m, const uint8_t *r, int n, const orc_scoring *sc,
                    orc_result *res)
{
    int *Hrow = malloc(sizeof(int) * (size_t)(n + 1));
    int *Frow = malloc(sizeof(int) * (size_t)(n + 1));
    score_linear(q, m, r, n, sc, res, Hrow, Frow);
    free(Hrow);
    free(Frow);
    return 0;
}

/* Full H, E, F matrices ((m+1) x (n+1), row-major) for invariant tests. */
int orc_matrices(const uint8_t *q, int m, const uint8_t *r, int n, const orc_scoring *sc,
                 int32_t *H, int32_t *E, int32_t *F)
{
    const int W = n + 1;
    for (int j = 0; j <= n; j++) {
        H[j] = 0;
        E[j] = NEG;
        F[j] = NEG;
    }
    for (int i = 1; i <= m; i++) {
        H[(size_t)i * W] = 0;
        E[(size_t)i * W] = NEG;
        F[(size_t)i * W] = NEG;
        for (int j = 1; j <= n; j++) {
            int s = (q[i - 1] == r[j - 1]) ? sc->match : sc->mismatch;
            int e = imax(H[(size_t)i * W + j - 1] + sc->gap_open, E[(size_t)i * W + j - 1] + sc->gap_extend);
            int f = imax(H[(size_t)(i - 1) * W + j] + sc->gap_open, F[(size_t)(i - 1) * W + j] + sc->gap_extend);
            int h = imax(imax(0, H[(size_t)(i - 1) * W + j - 1] + s), imax(e, f));
            E[(size_t)i * W + j] = e;
            F[(size_t)i * W + j] = f;
            H[(size_t)i * W + j] = h;
        }
    }
    return 0;
}
