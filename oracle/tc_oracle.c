/*
 * Plain FP64 CPU oracle for the general dense tensor contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the benchmark's
 * CPU baseline can compare the GPU path against an obviously correct loop nest.
 * It shares no code, header or helper with the GPU library.
 *
 * What it computes is the element-wise definition of the contraction
 * (Sec. 4, eq. gen-contraction), with the alpha/beta update of the
 * element-wise GEMM definition (Sec. 3) and arbitrary element strides for
 * every tensor dimension (Sec. 6.1, the generic-layout location formula):
 *
 *   C[f] := alpha * sum_{p} A[f|A, p] * B[f|B, p] + beta * C[f]
 *
 * where f runs over the labels of C and p over the labels shared by A and B.
 * Readings of points the paper leaves open:
 *   - beta == 0 means C is write-only (its old contents, NaN or not, are not
 *     read); alpha == 0 means A and B are not read at all and C := beta * C
 *     (the BLAS convention for the alpha/beta update of Sec. 3), so NaN or
 *     Inf in A or B do not reach C when alpha == 0.
 *   - a label must appear in exactly two of the three tensors, once each, with
 *     equal extents; anything else is rejected (no trace / batch indices).
 *   - the sum over p runs over every p in colexicographic order (first label
 *     of A's order fastest), multiply and add as separate roundings
 *     (compile with -ffp-contract=off), accumulated in double from zero.
 *
 * Parity status of each entry point is stated at its definition.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_MAXDIM 32

#define ORC_OK 0
#define ORC_ERR_NULL (-1)
#define ORC_ERR_NDIM (-2)
#define ORC_ERR_LABEL (-3)
#define ORC_ERR_EXTENT (-4)

/* One contraction problem after the labels have been resolved. */
typedef struct {
    int nf;                      /* labels of C (free indices), in C's order */
    int64_t flen[ORC_MAXDIM];
    int64_t fsC[ORC_MAXDIM];     /* stride in C */
    int64_t fsA[ORC_MAXDIM];     /* stride in A, 0 when the label is not in A */
    int64_t fsB[ORC_MAXDIM];     /* stride in B, 0 when the label is not in B */
    int np;                      /* contracted labels, in A's order */
    int64_t plen[ORC_MAXDIM];
    int64_t psA[ORC_MAXDIM];
    int64_t psB[ORC_MAXDIM];
} orc_problem;

static int find_label(char l, int nd, const char* idx) {
    for (int i = 0; i < nd; ++i)
        if (idx[i] == l) return i;
    return -1;
}

static int unique_labels(int nd, const char* idx) {
    for (int i = 0; i < nd; ++i)
        for (int j = i + 1; j < nd; ++j)
            if (idx[i] == idx[j]) return 0;
    return 1;
}

/* Resolve labels into free (C) and contracted (A and B) index lists. */
static int resolve(int ndA, const int64_t* lenA, const int64_t* strA, const char* idxA,
                   int ndB, const int64_t* lenB, const int64_t* strB, const char* idxB,
                   int ndC, const int64_t* lenC, const int64_t* strC, const char* idxC,
                   orc_problem* pr) {
    if (ndA < 0 || ndB < 0 || ndC < 0 || ndA > ORC_MAXDIM || ndB > ORC_MAXDIM || ndC > ORC_MAXDIM)
        return ORC_ERR_NDIM;
    if ((ndA && (!lenA || !strA || !idxA)) || (ndB && (!lenB || !strB || !idxB)) ||
        (ndC && (!lenC || !strC || !idxC)))
        return ORC_ERR_NULL;
    if (!unique_labels(ndA, idxA) || !unique_labels(ndB, idxB) || !unique_labels(ndC, idxC))
        return ORC_ERR_LABEL;

    pr->nf = 0;
    for (int c = 0; c < ndC; ++c) {
        int a = find_label(idxC[c], ndA, idxA);
        int b = find_label(idxC[c], ndB, idxB);
        if ((a >= 0) == (b >= 0)) return ORC_ERR_LABEL; /* in both or in neither */
        int64_t other = (a >= 0) ? lenA[a] : lenB[b];
        if (other != lenC[c]) return ORC_ERR_EXTENT;
        pr->flen[pr->nf] = lenC[c];
        pr->fsC[pr->nf] = strC[c];
        pr->fsA[pr->nf] = (a >= 0) ? strA[a] : 0;
        pr->fsB[pr->nf] = (b >= 0) ? strB[b] : 0;
        pr->nf++;
    }
    pr->np = 0;
    for (int a = 0; a < ndA; ++a) {
        int c = find_label(idxA[a], ndC, idxC);
        int b = find_label(idxA[a], ndB, idxB);
        if (c >= 0) continue; /* free index, handled above */
        if (b < 0) return ORC_ERR_LABEL;  /* only in A */
        if (lenB[b] != lenA[a]) return ORC_ERR_EXTENT;
        pr->plen[pr->np] = lenA[a];
        pr->psA[pr->np] = strA[a];
        pr->psB[pr->np] = strB[b];
        pr->np++;
    }
    for (int b = 0; b < ndB; ++b) {
        if (find_label(idxB[b], ndA, idxA) < 0 && find_label(idxB[b], ndC, idxC) < 0)
            return ORC_ERR_LABEL; /* only in B */
    }
    return ORC_OK;
}

static int64_t count_of(int n, const int64_t* len) {
    int64_t t = 1;
    for (int i = 0; i < n; ++i) t *= len[i];
    return t;
}

/* Split a colexicographic linear index into a multi-index (first fastest). */
static void unlinearize(int64_t lin, int n, const int64_t* len, int64_t* idx) {
    for (int i = 0; i < n; ++i) {
        idx[i] = lin % len[i];
        lin /= len[i];
    }
}

/*
 * The sum over the contracted indices for one output multi-index.
 * absval != 0 gives the contraction of |A| and |B| (used for error bounds).
 */
static double contracted_sum(const orc_problem* pr, const double* A, const double* B,
                             int64_t baseA, int64_t baseB, int absval) {
    int64_t nP = count_of(pr->np, pr->plen);
    int64_t p[ORC_MAXDIM];
    for (int i = 0; i < pr->np; ++i) p[i] = 0;
    double sum = 0.0;
    for (int64_t q = 0; q < nP; ++q) {
        int64_t offA = baseA, offB = baseB;
        for (int i = 0; i < pr->np; ++i) {
            offA += p[i] * pr->psA[i];
            offB += p[i] * pr->psB[i];
        }
        double a = A[offA], b = B[offB];
        if (absval) {
            a = fabs(a);
            b = fabs(b);
        }
        double prod = a * b;
        sum = sum + prod;
        /* advance p in colexicographic order */
        for (int i = 0; i < pr->np; ++i) {
            if (++p[i] < pr->plen[i]) break;
            p[i] = 0;
        }
    }
    return sum;
}

static double update(double alpha, double sum, double beta, double c0) {
    double r = alpha * sum;
    if (beta != 0.0) r = r + beta * c0;
    return r;
}

/* alpha == 0: the sum is not formed (A and B unread); C := beta * C. */
static double scale_only(double beta, double c0) {
    return beta != 0.0 ? beta * c0 : 0.0;
}

/*
 * Full contraction into C (host arrays, strides in elements).
 * Parity pinned in the test suite against: numpy.einsum, an explicit
 * transpose-transpose-GEMM-transpose route (Sec. 5, fig. TTGT), the identity
 * tensor, integer-exact inputs, linearity, label and storage permutations, and
 * the GEMM / dot / outer-product special cases.
 */
int oracle_contract(double alpha,
                    const double* A, int ndA, const int64_t* lenA, const int64_t* strA, const char* idxA,
                    const double* B, int ndB, const int64_t* lenB, const int64_t* strB, const char* idxB,
                    double beta,
                    double* C, int ndC, const int64_t* lenC, const int64_t* strC, const char* idxC,
                    int absval, int nthreads) {
    orc_problem pr;
    int st = resolve(ndA, lenA, strA, idxA, ndB, lenB, strB, idxB, ndC, lenC, strC, idxC, &pr);
    if (st != ORC_OK) return st;
    int64_t nF = count_of(pr.nf, pr.flen);
    if (nF == 0) return ORC_OK;
    if (!C || (alpha != 0.0 && count_of(pr.np, pr.plen) > 0 && (!A || !B))) return ORC_ERR_NULL;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t lin = 0; lin < nF; ++lin) {
        int64_t f[ORC_MAXDIM];
        unlinearize(lin, pr.nf, pr.flen, f);
        int64_t offC = 0, baseA = 0, baseB = 0;
        for (int i = 0; i < pr.nf; ++i) {
            offC += f[i] * pr.fsC[i];
            baseA += f[i] * pr.fsA[i];
            baseB += f[i] * pr.fsB[i];
        }
        if (alpha == 0.0) {
            C[offC] = scale_only(beta, beta != 0.0 ? C[offC] : 0.0);
            continue;
        }
        double s = contracted_sum(&pr, A, B, baseA, baseB, absval);
        C[offC] = update(alpha, s, beta, beta != 0.0 ? C[offC] : 0.0);
    }
    return ORC_OK;
}

/*
 * The same definition evaluated only at selected outputs: pts holds npts
 * multi-indices over C's labels (npts x ndC, row by row).  out[q] receives the
 * updated value C would hold at pts[q]; C itself is only read (for beta != 0).
 * Used to check full-size GPU results at sampled points.  Pinned by the test
 * that compares it with oracle_contract on every point of small problems.
 */
int oracle_contract_points(double alpha,
                           const double* A, int ndA, const int64_t* lenA, const int64_t* strA, const char* idxA,
                           const double* B, int ndB, const int64_t* lenB, const int64_t* strB, const char* idxB,
                           double beta,
                           const double* C, int ndC, const int64_t* lenC, const int64_t* strC, const char* idxC,
                           int64_t npts, const int64_t* pts, double* out, int absval, int nthreads) {
    orc_problem pr;
    int st = resolve(ndA, lenA, strA, idxA, ndB, lenB, strB, idxB, ndC, lenC, strC, idxC, &pr);
    if (st != ORC_OK) return st;
    if (npts > 0 && (!pts || !out)) return ORC_ERR_NULL;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t q = 0; q < npts; ++q) {
        const int64_t* f = pts + q * ndC;
        int64_t offC = 0, baseA = 0, baseB = 0;
        for (int i = 0; i < pr.nf; ++i) {
            offC += f[i] * pr.fsC[i];
            baseA += f[i] * pr.fsA[i];
            baseB += f[i] * pr.fsB[i];
        }
        const double c0 = (beta != 0.0 && C) ? C[offC] : 0.0;
        if (alpha == 0.0) {
            out[q] = scale_only(beta, c0);
            continue;
        }
        double s = contracted_sum(&pr, A, B, baseA, baseB, absval);
        out[q] = update(alpha, s, beta, c0);
    }
    return ORC_OK;
}
