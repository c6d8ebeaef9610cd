/*
 * ldpc_oracle.c -- plain CPU reference decoders.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is the oracle that the GPU decoders are checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product library never links or calls it.  It shares no code,
 * table or header with the GPU path.
 *
 * Everything is written the slow, obvious way:
 *   - GF(2^p) multiplication is carry-less polynomial multiplication reduced
 *     modulo the primitive polynomial (sec. 2.1: field elements are
 *     polynomials over GF(2); addition is XOR).  Inverses are found by search.
 *   - Non-binary decoding follows Alg. 2 (Min-Max) step by step: the forward
 *     and backward matrices of eqs. (7)-(10) are computed for every edge
 *     position exactly as written, including F at the last edge and B at the
 *     first edge, which the outputs never use; the beta messages follow eqs.
 *     (11)-(13) and the variable-node update eqs. (14)-(15).  Messages are
 *     int32; alpha is clamped when stored, to 32767 by default (a reading: the
 *     paper does not state a saturation) or to nb_msg_max for the reduced-precision
 *     variants of sec. 5 (8-bit messages: 127); the channel vector then takes part
 *     clipped to the same bound, gamma'(x) = min(gamma(x), nb_msg_max).  Ties in the
 *     hard decision go to the lowest x.  The layered Min-Max schedule (a reading; the
 *     paper describes the two-phase one only) runs the same check node one check at a
 *     time, in the order of orc_nb_layers, forming each incoming alpha from eq. (14)
 *     with the betas as they stand at that moment; decisions follow each full pass.
 *   - Binary min-sum is the GF(2) case of the same check-node rule written in
 *     the log-likelihood-ratio form: each outgoing message is the product of
 *     the other edges' signs times a normalised minimum of the other edges'
 *     magnitudes, found by a naive loop over the other edges (no min1/min2
 *     compression).  Normalisation: NMS (num * m) >> shift, OMS max(m - off, 0),
 *     MS m.  Flooding follows the two-phase schedule of Alg. 2; layered
 *     processes rows one at a time in ascending order.  In both schedules the
 *     check node sees the variable-to-check message saturated to +-msg_max,
 *     while the a posteriori sum Lambda = L + sum_m r_mn is kept exact (a
 *     reading: the paper does not define binary min-sum or its saturation).
 *   - Iteration semantics follow Alg. 2: iteration k first tests the syndrome
 *     of the decision of iteration k-1 and stops when it is zero (early stop),
 *     so a codeword whose channel decision already satisfies H is reported
 *     with 0 iterations.
 *
 * Parallelism: OpenMP over independent codewords only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <limits.h>

enum { ORC_MS = 0, ORC_NMS = 1, ORC_OMS = 2, ORC_MINMAX = 3 };
enum { ORC_FLOODING = 0, ORC_LAYERED = 1 };

typedef struct {
    int32_t max_iters;
    int32_t early_stop;
    int32_t schedule;
    int32_t rule;
    int32_t nms_num;
    int32_t nms_shift;
    int32_t oms_offset;
    int32_t msg_max;
    int32_t nb_msg_max; /* Min-Max message bound, 0 = 32767 */
} orc_params;

/* ------------------------------------------------------------------ GF(2^p) */

static int log2i(int g) { int p = 0; while ((1 << p) < g) p++; return p; }

int orc_gf_mul(int g, uint32_t poly, int a, int b)
{
    int p = log2i(g);
    uint32_t r = 0;
    for (int i = 0; i < p; i++)
        if ((b >> i) & 1) r ^= (uint32_t)a << i;
    for (int d = 2 * p - 2; d >= p; d--)
        if ((r >> d) & 1) r ^= poly << (d - p);
    return (int)r;
}

int orc_gf_inv(int g, uint32_t poly, int a)
{
    for (int b = 1; b < g; b++)
        if (orc_gf_mul(g, poly, a, b) == 1) return b;
    return 0;
}

/* out(x) = in(h^-1 x): the distribution of h*c when c is distributed as `in`
 * (multiplying a message by h, the permutation of sec. 2.2). */
void orc_gf_permute(int g, uint32_t poly, int h, const int32_t *in, int32_t *out)
{
    int hinv = orc_gf_inv(g, poly, h);
    for (int x = 0; x < g; x++) out[x] = in[orc_gf_mul(g, poly, hinv, x)];
}

/* 1 when sum_j h_{m,j} c_{col_j} = 0 (GF addition = XOR) for every check m. */
int orc_syndrome_ok(int g, uint32_t poly, int m, const int32_t *row_ptr, const int32_t *col_idx,
                    const uint8_t *h_val, const uint8_t *c)
{
    for (int i = 0; i < m; i++) {
        int s = 0;
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            int h = h_val ? h_val[e] : 1;
            s ^= orc_gf_mul(g, poly, h, c[col_idx[e]]);
        }
        if (s) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------ binary min-sum */

static int norm_mag(const orc_params *P, int mag)
{
    switch (P->rule) {
    case ORC_NMS: return (P->nms_num * mag) >> P->nms_shift;
    case ORC_OMS: return mag > P->oms_offset ? mag - P->oms_offset : 0;
    default: return mag;
    }
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Check-node rule for one check of degree dc: r_j = prod_{k!=j} sgn(q_k) * f(min_{k!=j} |q_k|),
 * with sgn(0) = +1. */
void orc_binary_cn(int dc, const int32_t *q, int32_t *r, const orc_params *P)
{
    for (int j = 0; j < dc; j++) {
        int mn = INT_MAX, neg = 0;
        for (int k = 0; k < dc; k++) {
            if (k == j) continue;
            int a = q[k] < 0 ? -q[k] : q[k];
            if (a < mn) mn = a;
            if (q[k] < 0) neg ^= 1;
        }
        int mag = norm_mag(P, mn);
        r[j] = neg ? -mag : mag;
    }
}

typedef struct {
    int n, m;
    const int32_t *row_ptr, *col_idx;
} bin_code;

static void bin_decide(int n, const int32_t *lam, uint8_t *hard)
{
    for (int v = 0; v < n; v++) hard[v] = lam[v] < 0;
}

static void bin_decode_one(const bin_code *C, const orc_params *P, const int8_t *L,
                           uint8_t *hard, int16_t *iters_out, uint8_t *ok_out,
                           int32_t *dq, int32_t *dr, int32_t *dlam)
{
    int n = C->n, m = C->m, E = C->row_ptr[m];
    int32_t *lam = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *r = (int32_t *)malloc(sizeof(int32_t) * (E ? E : 1));
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (E ? E : 1));
    int mm = P->msg_max;
    for (int v = 0; v < n; v++) lam[v] = L[v];
    for (int e = 0; e < E; e++) r[e] = 0;
    bin_decide(n, lam, hard);
    int it = 0;
    for (int k = 1; k <= P->max_iters; k++) {
        if (P->early_stop && orc_syndrome_ok(2, 0x3, m, C->row_ptr, C->col_idx, NULL, hard)) break;
        if (P->schedule == ORC_FLOODING) {
            /* check-node phase on the messages of iteration k-1 */
            for (int e = 0; e < E; e++) q[e] = clampi(lam[C->col_idx[e]] - r[e], -mm, mm);
            for (int i = 0; i < m; i++) {
                int b = C->row_ptr[i], dc = C->row_ptr[i + 1] - b;
                orc_binary_cn(dc, q + b, r + b, P);
            }
            /* variable-node phase: a posteriori sum */
            for (int v = 0; v < n; v++) lam[v] = L[v];
            for (int e = 0; e < E; e++) lam[C->col_idx[e]] += r[e];
        } else {
            /* Row-by-row: the check sees the saturated message clamp(Lambda - r_old); the
             * a posteriori value is updated exactly, Lambda <- Lambda - r_old + r_new, so
             * that Lambda = L + sum of the current check messages at every step. */
            for (int i = 0; i < m; i++) {
                int b = C->row_ptr[i], dc = C->row_ptr[i + 1] - b;
                for (int e = b; e < b + dc; e++) q[e] = clampi(lam[C->col_idx[e]] - r[e], -mm, mm);
                for (int e = b; e < b + dc; e++) lam[C->col_idx[e]] -= r[e];
                orc_binary_cn(dc, q + b, r + b, P);
                for (int e = b; e < b + dc; e++) lam[C->col_idx[e]] += r[e];
            }
        }
        bin_decide(n, lam, hard);
        it = k;
    }
    *iters_out = (int16_t)it;
    *ok_out = (uint8_t)orc_syndrome_ok(2, 0x3, m, C->row_ptr, C->col_idx, NULL, hard);
    if (dq) for (int e = 0; e < E; e++) dq[e] = clampi(lam[C->col_idx[e]] - r[e], -mm, mm);
    if (dr) for (int e = 0; e < E; e++) dr[e] = r[e];
    if (dlam) for (int v = 0; v < n; v++) dlam[v] = lam[v];
    free(lam); free(r); free(q);
}

/* Decode `batch` codewords.  llr: int8 [batch][n]; hard: uint8 [batch][n] (one bit per byte);
 * optional dumps (int32, may be NULL): q [batch][E], r [batch][E], lam [batch][n]. */
int orc_decode_binary(int n, int m, const int32_t *row_ptr, const int32_t *col_idx,
                      const orc_params *P, int batch, const int8_t *llr, uint8_t *hard,
                      uint8_t *syndrome_ok, int16_t *iters, int32_t *dump_q, int32_t *dump_r,
                      int32_t *dump_lam, int nthreads)
{
    for (int i = 0; i < m; i++)
        if (row_ptr[i + 1] - row_ptr[i] < 2) return -1;
    bin_code C = { n, m, row_ptr, col_idx };
    int E = row_ptr[m];
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < batch; b++) {
        bin_decode_one(&C, P, llr + (size_t)b * n, hard + (size_t)b * n, iters + b, syndrome_ok + b,
                       dump_q ? dump_q + (size_t)b * E : NULL, dump_r ? dump_r + (size_t)b * E : NULL,
                       dump_lam ? dump_lam + (size_t)b * n : NULL);
    }
    return 0;
}

/* -------------------------------------------------------- non-binary Min-Max */

#define BIG INT_MAX

/* Check-node processing of Alg. 2 for one check of degree dc over GF(g).
 * alpha: [dc][g] incoming messages indexed by symbol value; beta: [dc][g] out.
 * h: the dc nonzero coefficients in edge order.  *pairs (may be NULL) is
 * incremented by the number of (max, min) pairs evaluated in the forward,
 * backward and middle-beta loops. */
void orc_minmax_cn(int g, uint32_t poly, int dc, const uint8_t *h, const int32_t *alpha,
                   int32_t *beta, int64_t *pairs_fb, int64_t *pairs_beta)
{
    int32_t *F = (int32_t *)malloc(sizeof(int32_t) * dc * g);
    int32_t *B = (int32_t *)malloc(sizeof(int32_t) * dc * g);
    int64_t nfb = 0, nb = 0;
    /* eq. (7): F at the first edge is alpha at h^-1 x; eq. (8): B at the last edge likewise */
    int hinv0 = orc_gf_inv(g, poly, h[0]);
    int hinvl = orc_gf_inv(g, poly, h[dc - 1]);
    for (int x = 0; x < g; x++) {
        F[x] = alpha[orc_gf_mul(g, poly, hinv0, x)];
        B[(dc - 1) * g + x] = alpha[(dc - 1) * g + orc_gf_mul(g, poly, hinvl, x)];
    }
    /* eq. (9): F_n(x) = min over x' + h_n x'' = x of max(F_{n-1}(x'), alpha_n(x'')) */
    for (int j = 1; j < dc; j++) {
        int32_t *Fj = F + j * g;
        const int32_t *Fp = F + (j - 1) * g;
        const int32_t *a = alpha + j * g;
        for (int x = 0; x < g; x++) Fj[x] = BIG;
        for (int x1 = 0; x1 < g; x1++)
            for (int x2 = 0; x2 < g; x2++) {
                int x = x1 ^ orc_gf_mul(g, poly, h[j], x2);
                int v = Fp[x1] > a[x2] ? Fp[x1] : a[x2];
                if (v < Fj[x]) Fj[x] = v;
                nfb++;
            }
    }
    /* eq. (10): B_{n-1}(x) = min over x' + h_{n-1} x'' = x of max(B_n(x'), alpha_{n-1}(x'')) */
    for (int j = dc - 1; j >= 1; j--) {
        int32_t *Bo = B + (j - 1) * g;
        const int32_t *Bi = B + j * g;
        const int32_t *a = alpha + (j - 1) * g;
        for (int x = 0; x < g; x++) Bo[x] = BIG;
        for (int x1 = 0; x1 < g; x1++)
            for (int x2 = 0; x2 < g; x2++) {
                int x = x1 ^ orc_gf_mul(g, poly, h[j - 1], x2);
                int v = Bi[x1] > a[x2] ? Bi[x1] : a[x2];
                if (v < Bo[x]) Bo[x] = v;
                nfb++;
            }
    }
    /* eq. (11): first edge; eq. (12): last edge */
    for (int x = 0; x < g; x++) {
        beta[x] = B[1 * g + orc_gf_mul(g, poly, h[0], x)];
        beta[(dc - 1) * g + x] = F[(dc - 2) * g + orc_gf_mul(g, poly, h[dc - 1], x)];
    }
    /* eq. (13): middle edges, min over x' + h_n x = x'' of max(F_{n-1}(x''), B_{n+1}(x')) */
    for (int j = 1; j < dc - 1; j++) {
        int32_t *bo = beta + j * g;
        const int32_t *Fp = F + (j - 1) * g;
        const int32_t *Bn = B + (j + 1) * g;
        for (int x = 0; x < g; x++) {
            int best = BIG;
            int hx = orc_gf_mul(g, poly, h[j], x);
            for (int x1 = 0; x1 < g; x1++) {
                int x2 = x1 ^ hx;
                int v = Fp[x2] > Bn[x1] ? Fp[x2] : Bn[x1];
                if (v < best) best = v;
                nb++;
            }
            bo[x] = best;
        }
    }
    if (pairs_fb) *pairs_fb += nfb;
    if (pairs_beta) *pairs_beta += nb;
    free(F); free(B);
}

typedef struct {
    int g; uint32_t poly; int n, m;
    const int32_t *row_ptr, *col_idx;
    const uint8_t *h_val;
    const int32_t *vn_ptr, *vn_edge;   /* edges of each variable node */
    const int32_t *order;              /* layered schedule: checks in processing order */
} nb_code;

/* eq. (14) for one edge e: gamma of its variable plus the betas of the variable's
 * other edges, shifted to minimum 0 and clipped to amax.  ap: g ints of scratch. */
static void nb_alpha(const nb_code *C, const int16_t *gamma, const int32_t *beta, int e, int amax,
                     int32_t *ap, int32_t *out)
{
    int g = C->g, v = C->col_idx[e];
    for (int x = 0; x < g; x++) {
        int s = gamma[(size_t)v * g + x];
        for (int u = C->vn_ptr[v]; u < C->vn_ptr[v + 1]; u++)
            if (C->vn_edge[u] != e) s += beta[(size_t)C->vn_edge[u] * g + x];
        ap[x] = s;
    }
    int mn = ap[0];
    for (int x = 1; x < g; x++) if (ap[x] < mn) mn = ap[x];
    for (int x = 0; x < g; x++) {
        int a = ap[x] - mn;
        out[x] = a > amax ? amax : a;
    }
}

/* Layers of the layered Min-Max schedule (a reading: the paper describes only the
 * two-phase schedule).  Checks are taken in ascending index and each joins the
 * lowest layer holding no check that shares a variable with it; the schedule then
 * processes the checks one at a time, layer by layer, ascending within a layer.
 * Brute force over earlier checks.  Returns the number of layers. */
int orc_nb_layers(int m, const int32_t *row_ptr, const int32_t *col_idx, int32_t *layer_of)
{
    int nl = 0;
    for (int i = 0; i < m; i++) {
        int l = 0;
        for (;; l++) {
            int clash = 0;
            for (int j = 0; j < i && !clash; j++) {
                if (layer_of[j] != l) continue;
                for (int a = row_ptr[i]; a < row_ptr[i + 1] && !clash; a++)
                    for (int c = row_ptr[j]; c < row_ptr[j + 1]; c++)
                        if (col_idx[a] == col_idx[c]) { clash = 1; break; }
            }
            if (!clash) break;
        }
        layer_of[i] = l;
        if (l + 1 > nl) nl = l + 1;
    }
    return nl;
}

static void nb_decide(const nb_code *C, const int16_t *gamma, const int32_t *beta, uint8_t *hard)
{
    int g = C->g;
    int32_t *app = (int32_t *)malloc(sizeof(int32_t) * g);
    for (int v = 0; v < C->n; v++) {
        for (int x = 0; x < g; x++) app[x] = gamma[(size_t)v * g + x];
        for (int t = C->vn_ptr[v]; t < C->vn_ptr[v + 1]; t++) {
            int e = C->vn_edge[t];
            for (int x = 0; x < g; x++) app[x] += beta[(size_t)e * g + x];
        }
        int best = 0;
        for (int x = 1; x < g; x++) if (app[x] < app[best]) best = x;
        hard[v] = (uint8_t)best;
    }
    free(app);
}

static void nb_decode_one(const nb_code *C, const orc_params *P, const int16_t *gamma_in,
                          uint8_t *hard, int16_t *iters_out, uint8_t *ok_out,
                          int32_t *dalpha, int32_t *dbeta, int64_t *pairs)
{
    int g = C->g, n = C->n, m = C->m, E = C->row_ptr[m];
    size_t EG = (size_t)(E ? E : 1) * g;
    int32_t *alpha = (int32_t *)malloc(sizeof(int32_t) * EG);
    int32_t *beta = (int32_t *)calloc(EG, sizeof(int32_t));
    int32_t *ap = (int32_t *)malloc(sizeof(int32_t) * g);
    const int32_t *order = C->order;
    int64_t pfb = 0, pb = 0;
    /* the channel vectors, clipped to the message bound of the chosen precision */
    int amax = P->nb_msg_max > 0 ? P->nb_msg_max : 32767;
    int16_t *gclip = (int16_t *)malloc(sizeof(int16_t) * (size_t)(n ? n : 1) * g);
    for (size_t i = 0; i < (size_t)n * g; i++) gclip[i] = (int16_t)(gamma_in[i] > amax ? amax : gamma_in[i]);
    const int16_t *gamma = gclip;
    /* Alg. 2 initialisation: alpha^(0) = gamma */
    for (int e = 0; e < E; e++)
        for (int x = 0; x < g; x++) alpha[(size_t)e * g + x] = gamma[(size_t)C->col_idx[e] * g + x];
    /* decision of iteration 0: the most likely channel symbol */
    for (int v = 0; v < n; v++) {
        int best = 0;
        for (int x = 1; x < g; x++) if (gamma[(size_t)v * g + x] < gamma[(size_t)v * g + best]) best = x;
        hard[v] = (uint8_t)best;
    }
    int it = 0;
    for (int k = 1; k <= P->max_iters; k++) {
        if (P->early_stop && orc_syndrome_ok(g, C->poly, m, C->row_ptr, C->col_idx, C->h_val, hard)) break;
        if (P->schedule == ORC_LAYERED) {
            /* one check at a time in layer order: its incoming alphas are formed from the
             * betas as they stand (eq. (14)), then its betas are replaced */
            for (int q = 0; q < m; q++) {
                int i = order[q];
                int b = C->row_ptr[i], dc = C->row_ptr[i + 1] - b;
                for (int e = b; e < b + dc; e++) nb_alpha(C, gamma, beta, e, amax, ap, alpha + (size_t)e * g);
                orc_minmax_cn(g, C->poly, dc, C->h_val + b, alpha + (size_t)b * g, beta + (size_t)b * g, &pfb, &pb);
            }
        } else {
            for (int i = 0; i < m; i++) {
                int b = C->row_ptr[i], dc = C->row_ptr[i + 1] - b;
                orc_minmax_cn(g, C->poly, dc, C->h_val + b, alpha + (size_t)b * g, beta + (size_t)b * g, &pfb, &pb);
            }
            /* eq. (14) on every edge */
            for (int e = 0; e < E; e++) nb_alpha(C, gamma, beta, e, amax, ap, alpha + (size_t)e * g);
        }
        /* decision: the a posteriori step after eq. (15) */
        nb_decide(C, gamma, beta, hard);
        it = k;
    }
    *iters_out = (int16_t)it;
    *ok_out = (uint8_t)orc_syndrome_ok(g, C->poly, m, C->row_ptr, C->col_idx, C->h_val, hard);
    if (dalpha) memcpy(dalpha, alpha, sizeof(int32_t) * (size_t)E * g);
    if (dbeta) memcpy(dbeta, beta, sizeof(int32_t) * (size_t)E * g);
    if (pairs) { pairs[0] += pfb; pairs[1] += pb; }
    free(alpha); free(beta); free(ap); free(gclip);
}

/* gamma: int16 [batch][n][g]; hard: uint8 [batch][n]; dumps int32 [batch][E][g] (may be NULL);
 * pairs: int64[2] accumulated (F&B pairs, middle-beta pairs), may be NULL. */
int orc_decode_nb(int g, uint32_t poly, int n, int m, const int32_t *row_ptr, const int32_t *col_idx,
                  const uint8_t *h_val, const orc_params *P, int batch, const int16_t *gamma,
                  uint8_t *hard, uint8_t *syndrome_ok, int16_t *iters, int32_t *dump_alpha,
                  int32_t *dump_beta, int64_t *pairs, int nthreads)
{
    int E = row_ptr[m];
    for (int i = 0; i < m; i++)
        if (row_ptr[i + 1] - row_ptr[i] < 2) return -1;
    int32_t *vn_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *vn_edge = (int32_t *)malloc(sizeof(int32_t) * (E ? E : 1));
    int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    for (int e = 0; e < E; e++) vn_ptr[col_idx[e] + 1]++;
    for (int v = 0; v < n; v++) vn_ptr[v + 1] += vn_ptr[v];
    for (int e = 0; e < E; e++) { int v = col_idx[e]; vn_edge[vn_ptr[v] + fill[v]++] = e; }
    int32_t *layer_of = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    int nl = orc_nb_layers(m, row_ptr, col_idx, layer_of), q = 0;
    for (int l = 0; l < nl; l++)
        for (int i = 0; i < m; i++) if (layer_of[i] == l) order[q++] = i;
    nb_code C = { g, poly, n, m, row_ptr, col_idx, h_val, vn_ptr, vn_edge, order };
    int64_t tot[2] = { 0, 0 };
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < batch; b++) {
        int64_t pr[2] = { 0, 0 };
        nb_decode_one(&C, P, gamma + (size_t)b * n * g, hard + (size_t)b * n, iters + b, syndrome_ok + b,
                      dump_alpha ? dump_alpha + (size_t)b * E * g : NULL,
                      dump_beta ? dump_beta + (size_t)b * E * g : NULL, pr);
#pragma omp atomic
        tot[0] += pr[0];
#pragma omp atomic
        tot[1] += pr[1];
    }
    if (pairs) { pairs[0] += tot[0]; pairs[1] += tot[1]; }
    free(vn_ptr); free(vn_edge); free(fill); free(layer_of); free(order);
    return 0;
}

/* ------------------------------------------------ fixed-point FFT-SPA (Alg. 1) */
/*
 * Alg. 1 in the probability domain with fixed point Q24 (2^24 = probability 1),
 * for fields up to GF(256).  The paper runs it in floating point and in 32- and
 * 8-bit fixed point without stating the fixed-point rules; these are the readings
 * used here:
 *   - channel: p~(x) = W(gamma(x)) with W(c) = round(2^24 exp(-c / 4)) (gamma is the
 *     symbol cost in units of a quarter LLR, so exp(-gamma/4) is proportional to
 *     p(c_n = x | y_n)), then p = norm(p~);
 *   - norm(z): with S = sum_x z(x) > 0 and R = floor(2^46 / S),
 *     norm(z)(x) = floor((z(x) R + 2^21) / 2^22); when S = 0 the result is the
 *     channel vector p_n (uniform 2^24 / g for the channel itself);
 *   - product of two Q24 numbers: qmul(a, b) = floor((a b + 2^23) / 2^24), applied in
 *     ascending edge order (the first factor taken as is);
 *   - eq. (3): the transform over GF(2^q) is the Walsh-Hadamard transform
 *     F(f) = sum_t (-1)^popcount(f & t) u(t), exact in integers; the inverse is the same
 *     sum, taken in 64 bits (its magnitude reaches g 2^24, beyond 32 bits from GF(128)
 *     on), followed by floor division by g and a clamp at 0;
 *   - permutation (eq. (2)) u'(t) = u(h^-1 t) and depermutation (eq. (4)) v'(x) = v(h x), as in
 *     the Min-Max reading (the distribution of h c_n);
 *   - eqs. (5)-(6): z(x) = qmul-product of p_n(x) and the other incoming v'; the
 *     outgoing message is norm(z);
 *   - decision: argmax of p_n(x) times every incoming v' (same product rule), lowest
 *     x on ties; the stop rule and iteration count are those of Alg. 2.
 */
#include <math.h>

#define SPA_Q 24

int orc_spa_weight(int c)
{
    if (c < 0) c = 0;
    return (int)floor((double)(1 << SPA_Q) * exp(-(double)c / 4.0) + 0.5);
}

static int64_t floordiv(int64_t x, int64_t d) { return x >= 0 ? x / d : -((-x + d - 1) / d); }

int32_t orc_spa_qmul(int32_t a, int32_t b)
{
    return (int32_t)floordiv((int64_t)a * b + ((int64_t)1 << (SPA_Q - 1)), (int64_t)1 << SPA_Q);
}

/* norm(z) into out; returns 0 when sum z = 0 (out untouched) */
int orc_spa_norm(int g, const int32_t *z, int32_t *out)
{
    int64_t s = 0;
    for (int x = 0; x < g; x++) s += z[x];
    if (s <= 0) return 0;
    int64_t r = ((int64_t)1 << 46) / s;
    for (int x = 0; x < g; x++) out[x] = (int32_t)(((int64_t)z[x] * r + ((int64_t)1 << 21)) >> 22);
    return 1;
}

static int popc(unsigned v) { int c = 0; while (v) { c += v & 1u; v >>= 1; } return c; }

/* out(f) = sum_t (-1)^popcount(f & t) in(t), in 64 bits */
static void wht64(int g, const int32_t *in, int64_t *out)
{
    for (int f = 0; f < g; f++) {
        int64_t s = 0;
        for (int t = 0; t < g; t++) s += (popc((unsigned)(f & t)) & 1) ? -(int64_t)in[t] : in[t];
        out[f] = s;
    }
}

/* The same transform with 32-bit outputs (every caller's sums fit 32 bits). */
void orc_wht(int g, const int32_t *in, int32_t *out)
{
    int64_t *w = (int64_t *)malloc(sizeof(int64_t) * g);
    wht64(g, in, w);
    for (int f = 0; f < g; f++) out[f] = (int32_t)w[f];
    free(w);
}

/* Check-node processing of Alg. 1 for one check: u: [dc][g] incoming Q24 messages,
 * v: [dc][g] outgoing (depermuted) messages. */
void orc_spa_cn(int g, uint32_t poly, int dc, const uint8_t *h, const int32_t *u, int32_t *v)
{
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)dc * g);
    int32_t *t1 = (int32_t *)malloc(sizeof(int32_t) * g);
    int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * g);
    int32_t *vv = (int32_t *)malloc(sizeof(int32_t) * g);
    int64_t *inv = (int64_t *)malloc(sizeof(int64_t) * g);
    for (int j = 0; j < dc; j++) {
        orc_gf_permute(g, poly, h[j], u + (size_t)j * g, t1);   /* eq. (2) */
        orc_wht(g, t1, U + (size_t)j * g);                      /* forward transform of eq. (3) */
    }
    for (int n = 0; n < dc; n++) {
        int first = 1;
        for (int j = 0; j < dc; j++) {
            if (j == n) continue;
            for (int f = 0; f < g; f++)
                acc[f] = first ? U[(size_t)j * g + f] : orc_spa_qmul(acc[f], U[(size_t)j * g + f]);
            first = 0;
        }
        wht64(g, acc, inv);                                     /* inverse transform */
        for (int t = 0; t < g; t++) {
            int64_t x = floordiv(inv[t], g);
            vv[t] = x < 0 ? 0 : (int32_t)x;
        }
        for (int x = 0; x < g; x++)                              /* eq. (4): v'(x) = v(h x) */
            v[(size_t)n * g + x] = vv[orc_gf_mul(g, poly, h[n], x)];
    }
    free(U); free(t1); free(acc); free(vv); free(inv);
}

static void spa_channel(int g, const int16_t *gam, int32_t *p)
{
    int32_t *w = (int32_t *)malloc(sizeof(int32_t) * g);
    for (int x = 0; x < g; x++) w[x] = orc_spa_weight(gam[x]);
    if (!orc_spa_norm(g, w, p))
        for (int x = 0; x < g; x++) p[x] = (1 << SPA_Q) / g;
    free(w);
}

static void spa_decode_one(const nb_code *C, const orc_params *P, const int16_t *gamma,
                           uint8_t *hard, int16_t *iters_out, uint8_t *ok_out, int32_t *du, int32_t *dv)
{
    int g = C->g, n = C->n, m = C->m, E = C->row_ptr[m];
    size_t EG = (size_t)(E ? E : 1) * g;
    int32_t *pch = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1) * g);
    int32_t *u = (int32_t *)malloc(sizeof(int32_t) * EG);
    int32_t *v = (int32_t *)calloc(EG, sizeof(int32_t));
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * g);
    for (int i = 0; i < n; i++) spa_channel(g, gamma + (size_t)i * g, pch + (size_t)i * g);
    for (int e = 0; e < E; e++)                                  /* initialisation: u = p */
        for (int x = 0; x < g; x++) u[(size_t)e * g + x] = pch[(size_t)C->col_idx[e] * g + x];
    for (int i = 0; i < n; i++) {
        int best = 0;
        for (int x = 1; x < g; x++) if (pch[(size_t)i * g + x] > pch[(size_t)i * g + best]) best = x;
        hard[i] = (uint8_t)best;
    }
    int it = 0;
    for (int k = 1; k <= P->max_iters; k++) {
        if (P->early_stop && orc_syndrome_ok(g, C->poly, m, C->row_ptr, C->col_idx, C->h_val, hard)) break;
        for (int i = 0; i < m; i++) {
            int b = C->row_ptr[i], dc = C->row_ptr[i + 1] - b;
            orc_spa_cn(g, C->poly, dc, C->h_val + b, u + (size_t)b * g, v + (size_t)b * g);
        }
        for (int i = 0; i < n; i++) {
            for (int t = C->vn_ptr[i]; t < C->vn_ptr[i + 1]; t++) {
                int e = C->vn_edge[t];
                for (int x = 0; x < g; x++) {
                    int32_t a = pch[(size_t)i * g + x];
                    for (int w = C->vn_ptr[i]; w < C->vn_ptr[i + 1]; w++)
                        if (w != t) a = orc_spa_qmul(a, v[(size_t)C->vn_edge[w] * g + x]);
                    z[x] = a;
                }
                if (!orc_spa_norm(g, z, u + (size_t)e * g))
                    for (int x = 0; x < g; x++) u[(size_t)e * g + x] = pch[(size_t)i * g + x];
            }
            /* a posteriori product and decision */
            int best = 0, bv = -1;
            for (int x = 0; x < g; x++) {
                int32_t a = pch[(size_t)i * g + x];
                for (int w = C->vn_ptr[i]; w < C->vn_ptr[i + 1]; w++) a = orc_spa_qmul(a, v[(size_t)C->vn_edge[w] * g + x]);
                if (a > bv) { bv = a; best = x; }
            }
            hard[i] = (uint8_t)best;
        }
        it = k;
    }
    *iters_out = (int16_t)it;
    *ok_out = (uint8_t)orc_syndrome_ok(g, C->poly, m, C->row_ptr, C->col_idx, C->h_val, hard);
    if (du) memcpy(du, u, sizeof(int32_t) * (size_t)E * g);
    if (dv) memcpy(dv, v, sizeof(int32_t) * (size_t)E * g);
    free(pch); free(u); free(v); free(z);
}

/* gamma: int16 [batch][n][g], g <= 256; hard: uint8 [batch][n]; dumps int32 [batch][E][g]
 * (may be NULL): u (variable-to-check) and v' (check-to-variable) messages in Q24. */
int orc_decode_spa(int g, uint32_t poly, int n, int m, const int32_t *row_ptr, const int32_t *col_idx,
                   const uint8_t *h_val, const orc_params *P, int batch, const int16_t *gamma,
                   uint8_t *hard, uint8_t *syndrome_ok, int16_t *iters, int32_t *dump_u,
                   int32_t *dump_v, int nthreads)
{
    int E = row_ptr[m];
    if (g > 256) return -2;
    for (int i = 0; i < m; i++)
        if (row_ptr[i + 1] - row_ptr[i] < 2) return -1;
    int32_t *vn_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *vn_edge = (int32_t *)malloc(sizeof(int32_t) * (E ? E : 1));
    int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    for (int e = 0; e < E; e++) vn_ptr[col_idx[e] + 1]++;
    for (int i = 0; i < n; i++) vn_ptr[i + 1] += vn_ptr[i];
    for (int e = 0; e < E; e++) { int i = col_idx[e]; vn_edge[vn_ptr[i] + fill[i]++] = e; }
    nb_code C = { g, poly, n, m, row_ptr, col_idx, h_val, vn_ptr, vn_edge };
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < batch; b++)
        spa_decode_one(&C, P, gamma + (size_t)b * n * g, hard + (size_t)b * n, iters + b, syndrome_ok + b,
                       dump_u ? dump_u + (size_t)b * E * g : NULL, dump_v ? dump_v + (size_t)b * E * g : NULL);
    free(vn_ptr); free(vn_edge); free(fill);
    return 0;
}
