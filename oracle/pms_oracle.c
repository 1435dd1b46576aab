/*
 * pms_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously correct CPU oracle for the planted (l, d) motif
 * set.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg load it.  It shares no code, table or encoding with the GPU library:
 * it compares characters, one position at a time.
 *
 * What it computes (Section I.A problem statement; Section III.A, the
 * enhanced brute force):
 *   Sigma = {A, C, G, T};  W_i = every length-l substring of sequence i, at
 *   each start 0 .. t-l, i.e. t-l+1 windows;  d_H = number of positions whose
 *   bases differ;  an l-mer x matches a window w when d_H(x, w) <= d.
 *   M = { x in Sigma^l : every sequence i has some window w in W_i with
 *         d_H(x, w) <= d },
 *   reported in ascending order of the candidate number defined below.
 *
 * Candidate numbering (Section IV.A hands each worker the number of its first
 * and last l-mer and generates l-mers on the fly): candidate k in [0, 4^l)
 * is the l-mer whose base p (p = 0 is the leftmost base) is base-4 digit
 * l-1-p of k, with A=0, C=1, G=2, T=3.  Ascending k is therefore the
 * dictionary order of the l-mer strings.
 *
 * Modes:
 *   ORACLE_BRUTE (0): unpruned.  Every candidate is compared with every
 *       window of every sequence, and only then is the decision taken.
 *   ORACLE_SKIP  (1): the enhanced rule of Section III.A: the first sequence
 *       with no matching window rejects the candidate and the remaining
 *       sequences are not examined.  It also counts the sequence visits so
 *       that the algorithmic compare count of the enhanced method is known.
 *
 * Threads split [k_begin, k_end) into contiguous index ranges, one per
 * thread, as the paper's workers split the l-mer numbers (Section IV.A).
 * Each range's motifs are ascending; concatenating in range order keeps the
 * whole list ascending.
 */
#include <ctype.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_BRUTE 0
#define ORACLE_SKIP 1

#define ORACLE_OK 0
#define ORACLE_ERR_ARGS (-1)
#define ORACLE_ERR_BYTE (-2)
#define ORACLE_ERR_NOMEM (-3)

static const char kBase[4] = {'A', 'C', 'G', 'T'};

/* Candidate k written out as l characters (first base = most significant
 * base-4 digit). */
static void decode_candidate(uint64_t k, int l, char *x) {
    for (int p = 0; p < l; ++p)
        x[p] = kBase[(k >> (2 * (l - 1 - p))) & 3u];
}

/* Smallest Hamming distance between x and any of the t-l+1 windows of s.
 * mism[j] accumulates the mismatches of window j position by position. */
static int seq_min_distance(const char *s, int t, int l, const char *x,
                            uint8_t *mism) {
    const int nw = t - l + 1;
    memset(mism, 0, (size_t)nw);
    for (int p = 0; p < l; ++p) {
        const char xp = x[p];
        const char *sp = s + p;
        for (int j = 0; j < nw; ++j)
            mism[j] += (uint8_t)(sp[j] != xp);
    }
    int best = l + 1;
    for (int j = 0; j < nw; ++j)
        if (mism[j] < best) best = mism[j];
    return best;
}

typedef struct {
    const char *seqs; /* n rows of t upper-case bytes */
    int n, t, l, d, mode;
    uint64_t k_begin, k_end;
    uint32_t *found; /* ascending candidate numbers of this range */
    uint64_t nfound, capfound;
    uint64_t visits; /* sequence scans performed (skip mode counts them) */
    int err;
} range_job;

static void *run_range(void *arg) {
    range_job *job = (range_job *)arg;
    const int n = job->n, t = job->t, l = job->l, d = job->d;
    uint8_t *mism = (uint8_t *)malloc((size_t)(t - l + 1));
    if (!mism) {
        job->err = ORACLE_ERR_NOMEM;
        return NULL;
    }
    char x[32];
    for (uint64_t k = job->k_begin; k < job->k_end; ++k) {
        decode_candidate(k, l, x);
        int accepted = 1;
        for (int i = 0; i < n; ++i) {
            const int m = seq_min_distance(job->seqs + (size_t)i * t, t, l, x, mism);
            job->visits += 1;
            if (m > d) {
                accepted = 0;
                if (job->mode == ORACLE_SKIP) break; /* the enhanced rule */
            }
        }
        if (!accepted) continue;
        if (job->nfound == job->capfound) {
            uint64_t nc = job->capfound ? 2 * job->capfound : 1024;
            uint32_t *nb = (uint32_t *)realloc(job->found, nc * sizeof(uint32_t));
            if (!nb) {
                job->err = ORACLE_ERR_NOMEM;
                break;
            }
            job->found = nb;
            job->capfound = nc;
        }
        job->found[job->nfound++] = (uint32_t)k;
    }
    free(mism);
    return NULL;
}

/* Copies the rows to upper case and checks every byte is a base. */
static int normalise(const char *seqs, int n, int t, char **out) {
    char *buf = (char *)malloc((size_t)n * t);
    if (!buf) return ORACLE_ERR_NOMEM;
    for (size_t q = 0; q < (size_t)n * t; ++q) {
        const char c = (char)toupper((unsigned char)seqs[q]);
        if (c != 'A' && c != 'C' && c != 'G' && c != 'T') {
            free(buf);
            return ORACLE_ERR_BYTE;
        }
        buf[q] = c;
    }
    *out = buf;
    return ORACLE_OK;
}

/*
 * oracle_solve: motifs among candidates [k_begin, k_end).
 *   seqs     n*t bytes, row-major, A/C/G/T in either case.
 *   out      room for cap candidate numbers; the smallest min(cap, count)
 *            motifs are written ascending.
 *   count    receives the number of motifs in the range.
 *   visits   optional: receives the number of (candidate, sequence) scans
 *            performed; in skip mode, times t-l+1, it is the algorithmic
 *            window-compare count of the enhanced brute force.
 * Returns ORACLE_OK or a negative error code.
 */
int oracle_solve(const char *seqs, int n, int t, int l, int d, uint64_t k_begin,
                 uint64_t k_end, int mode, int threads, uint32_t *out,
                 uint64_t cap, uint64_t *count, uint64_t *visits) {
    if (!seqs || !count || n < 1 || l < 1 || l > 16 || d < 0 || d > l || t < l)
        return ORACLE_ERR_ARGS;
    if (mode != ORACLE_BRUTE && mode != ORACLE_SKIP) return ORACLE_ERR_ARGS;
    const uint64_t total = 1ull << (2 * l);
    if (k_begin > k_end || k_end > total) return ORACLE_ERR_ARGS;
    if (cap > 0 && !out) return ORACLE_ERR_ARGS;
    if (threads < 1) threads = 1;
    const uint64_t span = k_end - k_begin;
    if ((uint64_t)threads > span && span > 0) threads = (int)span;

    char *up = NULL;
    int rc = normalise(seqs, n, t, &up);
    if (rc != ORACLE_OK) return rc;

    range_job *jobs = (range_job *)calloc((size_t)threads, sizeof(range_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(up);
        free(jobs);
        free(tids);
        return ORACLE_ERR_NOMEM;
    }
    for (int w = 0; w < threads; ++w) {
        jobs[w].seqs = up;
        jobs[w].n = n;
        jobs[w].t = t;
        jobs[w].l = l;
        jobs[w].d = d;
        jobs[w].mode = mode;
        jobs[w].k_begin = k_begin + span * (uint64_t)w / (uint64_t)threads;
        jobs[w].k_end = k_begin + span * (uint64_t)(w + 1) / (uint64_t)threads;
    }
    int started = 0;
    for (int w = 1; w < threads; ++w) {
        if (pthread_create(&tids[w], NULL, run_range, &jobs[w]) != 0) break;
        started = w;
    }
    run_range(&jobs[0]);
    for (int w = 1; w <= started; ++w) pthread_join(tids[w], NULL);
    for (int w = started + 1; w < threads; ++w) run_range(&jobs[w]);

    uint64_t total_found = 0, total_visits = 0;
    rc = ORACLE_OK;
    for (int w = 0; w < threads; ++w) {
        if (jobs[w].err) rc = jobs[w].err;
        for (uint64_t q = 0; q < jobs[w].nfound; ++q) {
            if (total_found < cap) out[total_found] = jobs[w].found[q];
            ++total_found;
        }
        total_visits += jobs[w].visits;
        free(jobs[w].found);
    }
    *count = total_found;
    if (visits) *visits = total_visits;
    free(jobs);
    free(tids);
    free(up);
    return rc;
}

/*
 * oracle_candidate_distances: for one candidate number, the smallest Hamming
 * distance to a window of each sequence (per_seq[i], i < n).  The candidate
 * is a motif exactly when every entry is <= d.  Used to check sampled
 * candidates one by one at sizes where a full sweep is too slow.
 */
int oracle_candidate_distances(const char *seqs, int n, int t, int l,
                               uint64_t k, int32_t *per_seq) {
    if (!seqs || !per_seq || n < 1 || l < 1 || l > 16 || t < l) return ORACLE_ERR_ARGS;
    if (k >= (1ull << (2 * l))) return ORACLE_ERR_ARGS;
    char *up = NULL;
    int rc = normalise(seqs, n, t, &up);
    if (rc != ORACLE_OK) return rc;
    uint8_t *mism = (uint8_t *)malloc((size_t)(t - l + 1));
    if (!mism) {
        free(up);
        return ORACLE_ERR_NOMEM;
    }
    char x[32];
    decode_candidate(k, l, x);
    for (int i = 0; i < n; ++i)
        per_seq[i] = seq_min_distance(up + (size_t)i * t, t, l, x, mism);
    free(mism);
    free(up);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Rows of their own lengths, N masking and both strands.
 *
 * Section VI (Conclusion) names larger and real sequence data as future work.
 * This oracle takes that reading: sequence i has its own length
 * t_i, and its window set is written out explicitly,
 *   W_i = { s_i[j .. j+l-1] : 0 <= j <= t_i - l, and, with ORACLE_MASK_N,
 *           no byte N/n inside }
 *         united, with ORACLE_BOTH, with { revcomp(w) : w in that set },
 * where revcomp reads w backwards and exchanges A<->T and C<->G.  M is the
 * same definition as above over these sets; a sequence whose set is empty
 * makes M empty.
 * ------------------------------------------------------------------------ */
#define ORACLE_MASK_N 1
#define ORACLE_BOTH 2

static char complement(char c) {
    switch (c) {
        case 'A': return 'T';
        case 'C': return 'G';
        case 'G': return 'C';
        default: return 'A'; /* 'T' */
    }
}

/* Smallest Hamming distance between x and the nw windows wins[j*l .. j*l+l). */
static int set_min_distance(const char *wins, int nw, int l, const char *x, uint8_t *mism) {
    memset(mism, 0, (size_t)nw);
    for (int p = 0; p < l; ++p) {
        const char xc = x[p];
        for (int j = 0; j < nw; ++j)
            mism[j] += (uint8_t)(wins[(size_t)j * l + p] != xc);
    }
    int lowest = l + 1;
    for (int j = 0; j < nw; ++j)
        if (mism[j] < lowest) lowest = mism[j];
    return lowest;
}

typedef struct {
    char **wins; /* per sequence: its window set, wcount[i] windows of l bytes */
    const int *wcount;
    int n, l, d, mode, max_w;
    uint64_t k_begin, k_end;
    uint32_t *found;
    uint64_t nfound, capfound;
    uint64_t visits;
    int err;
} range_job_ex;

static void *run_range_ex(void *arg) {
    range_job_ex *job = (range_job_ex *)arg;
    const int n = job->n, l = job->l, d = job->d;
    uint8_t *mism = (uint8_t *)malloc((size_t)job->max_w);
    if (!mism) {
        job->err = ORACLE_ERR_NOMEM;
        return NULL;
    }
    char x[32];
    for (uint64_t k = job->k_begin; k < job->k_end; ++k) {
        decode_candidate(k, l, x);
        int ok = 1;
        for (int i = 0; i < n; ++i) {
            const int m = set_min_distance(job->wins[i], job->wcount[i], l, x, mism);
            job->visits += 1;
            if (d < m) {
                ok = 0;
                if (job->mode == ORACLE_SKIP) break; /* the enhanced rule, extended inputs */
            }
        }
        if (!ok) continue;
        if (job->nfound == job->capfound) {
            uint64_t nc = job->capfound ? 2 * job->capfound : 1024;
            uint32_t *nb = (uint32_t *)realloc(job->found, nc * sizeof(uint32_t));
            if (!nb) {
                job->err = ORACLE_ERR_NOMEM;
                break;
            }
            job->found = nb;
            job->capfound = nc;
        }
        job->found[job->nfound++] = (uint32_t)k;
    }
    free(mism);
    return NULL;
}

/* Window set of one row (upper-cased), as defined above.  *out holds
 * *count windows of l bytes each. */
static int row_windows(const char *row, int t, int l, int flags, char **out, int *count) {
    char *up = (char *)malloc((size_t)t + 1);
    if (!up) return ORACLE_ERR_NOMEM;
    for (int q = 0; q < t; ++q) {
        const char c = (char)toupper((unsigned char)row[q]);
        const int base = c == 'A' || c == 'C' || c == 'G' || c == 'T';
        if (!base && !(c == 'N' && (flags & ORACLE_MASK_N))) {
            free(up);
            return ORACLE_ERR_BYTE;
        }
        up[q] = c;
    }
    const int nstarts = t - l + 1;
    const int per = (flags & ORACLE_BOTH) ? 2 : 1;
    char *w = (char *)malloc((size_t)nstarts * per * l + 1);
    if (!w) {
        free(up);
        return ORACLE_ERR_NOMEM;
    }
    int k = 0;
    for (int j = 0; j < nstarts; ++j) {
        int has_n = 0;
        for (int p = 0; p < l; ++p) has_n |= up[j + p] == 'N';
        if (has_n) continue;
        memcpy(w + (size_t)k * l, up + j, (size_t)l);
        ++k;
    }
    const int fwd = k;
    if (flags & ORACLE_BOTH)
        for (int q = 0; q < fwd; ++q) {
            for (int p = 0; p < l; ++p) w[(size_t)k * l + p] = complement(w[(size_t)q * l + l - 1 - p]);
            ++k;
        }
    free(up);
    *out = w;
    *count = k;
    return ORACLE_OK;
}

/*
 * oracle_solve_ex: motifs among candidates [k_begin, k_end) for n rows of
 * their own lengths (rows[i] has lengths[i] bytes) under `flags`.  Other
 * arguments and results as for oracle_solve; in skip mode `visits` counts the
 * (candidate, sequence) scans.
 */
int oracle_solve_ex(const char *const *rows, const int *lengths, int n, int l, int d, int flags,
                    uint64_t k_begin, uint64_t k_end, int mode, int threads, uint32_t *out,
                    uint64_t cap, uint64_t *count, uint64_t *visits) {
    if (!rows || !lengths || !count || n < 1 || l < 1 || l > 16 || d < 0 || d > l)
        return ORACLE_ERR_ARGS;
    if (mode != ORACLE_BRUTE && mode != ORACLE_SKIP) return ORACLE_ERR_ARGS;
    if (flags & ~(ORACLE_MASK_N | ORACLE_BOTH)) return ORACLE_ERR_ARGS;
    const uint64_t total = 1ull << (2 * l);
    if (k_begin > k_end || k_end > total) return ORACLE_ERR_ARGS;
    if (cap > 0 && !out) return ORACLE_ERR_ARGS;
    for (int i = 0; i < n; ++i)
        if (!rows[i] || lengths[i] < l) return ORACLE_ERR_ARGS;
    if (threads < 1) threads = 1;
    const uint64_t span = k_end - k_begin;
    if ((uint64_t)threads > span && span > 0) threads = (int)span;

    char **wins = (char **)calloc((size_t)n, sizeof(char *));
    int *wcount = (int *)calloc((size_t)n, sizeof(int));
    if (!wins || !wcount) {
        free(wins);
        free(wcount);
        return ORACLE_ERR_NOMEM;
    }
    int rc = ORACLE_OK, max_w = 1, empty = 0;
    for (int i = 0; i < n && rc == ORACLE_OK; ++i) {
        rc = row_windows(rows[i], lengths[i], l, flags, &wins[i], &wcount[i]);
        if (rc == ORACLE_OK) {
            if (wcount[i] > max_w) max_w = wcount[i];
            if (wcount[i] == 0) empty = 1;
        }
    }
    uint64_t total_found = 0, total_visits = 0;
    if (rc == ORACLE_OK && !empty) {
        range_job_ex *jobs = (range_job_ex *)calloc((size_t)threads, sizeof(range_job_ex));
        pthread_t *tids = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
        if (!jobs || !tids) {
            rc = ORACLE_ERR_NOMEM;
        } else {
            for (int w = 0; w < threads; ++w) {
                jobs[w].wins = wins;
                jobs[w].wcount = wcount;
                jobs[w].n = n;
                jobs[w].l = l;
                jobs[w].d = d;
                jobs[w].mode = mode;
                jobs[w].max_w = max_w;
                jobs[w].k_begin = k_begin + (uint64_t)w * span / (uint64_t)threads;
                jobs[w].k_end = k_begin + (uint64_t)(w + 1) * span / (uint64_t)threads;
            }
            int started = 0;
            for (int w = 1; w < threads; ++w) {
                if (pthread_create(&tids[w], NULL, run_range_ex, &jobs[w]) != 0) break;
                started = w;
            }
            run_range_ex(&jobs[0]);
            for (int w = 1; w <= started; ++w) pthread_join(tids[w], NULL);
            for (int w = started + 1; w < threads; ++w) run_range_ex(&jobs[w]);
            for (int w = 0; w < threads; ++w) {
                if (jobs[w].err) rc = jobs[w].err;
                for (uint64_t q = 0; q < jobs[w].nfound; ++q) {
                    if (total_found < cap) out[total_found] = jobs[w].found[q];
                    ++total_found;
                }
                total_visits += jobs[w].visits;
                free(jobs[w].found);
            }
        }
        free(jobs);
        free(tids);
    }
    for (int i = 0; i < n; ++i) free(wins[i]);
    free(wins);
    free(wcount);
    *count = total_found;
    if (visits) *visits = total_visits;
    return rc;
}
