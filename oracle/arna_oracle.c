/*
 * arna_oracle.c -- FP64 CPU oracle for one SIR iteration with RNA / ARNA
 * distributed resampling (Demirel, Smal, Niessen, Meijering, Sbalzarini,
 * "An Adaptive Distributed Resampling Algorithm with Non-Proportional
 * Allocation", arXiv:1310.4624).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, calls or falls back to it.  It shares no source with the HIP code.
 *
 * Everything is double precision.  Each step of Alg. 3 (ARNA; Alg. 2 for RNA)
 * is written out in the paper's order:
 *   1  randomize the ring (Fisher-Yates, Sec. IV-B)            -> orc_ring
 *   2  exchange ratio from PE_eff (Eq. 3, Eq. 4)                -> orc_nex
 *   3  exchange N_ex particles with the ring neighbour (III-A/C) -> exchange map
 *   4  renormalize the carried weights by W_{k-1}
 *   5  (P) propagate and (U) update with the likelihood (Alg. 1)
 *   6  per-PE estimate x^m_k and weight sum W^(m)_k
 *   7  local systematic resampling (Alg. 1, last line)           -> orc_resample
 *   8  every particle of PE m carries W^(m)_k
 *   9-10 master: global estimate x_k, W_k (and the PE masses for Eq. 4)
 *
 * Points the paper leaves open are fixed as follows (the same readings are
 * listed in the design notes next to the GPU code):
 *   - PE_eff is the effective number of PEs, (sum_m W_m)^2 / sum_m W_m^2, in
 *     [1, M]; it is evaluated on integer PE masses P_m = floor(e^{L_m-Lmax} 2^20).
 *   - N_ex = floor(N_p (M D - S^2) / (2 (M-1) D)) with S = sum P, D = sum P^2
 *     (Eq. 3 with PE_eff = S^2/D); zero when PE_eff > cutoff * M (tracking
 *     benchmark text: no exchange above 99%); zero when M = 1; the first
 *     iteration uses the initial ratio; RNA uses floor(r N_p).
 *   - The N_ex particles a PE sends are chosen by systematic selection with a
 *     random offset c_m; received particles fill the vacated slots.
 *   - Systematic resampling runs on 32-bit fixed-point weights Q_i.
 *   - The likelihood is the Gaussian log-likelihood ratio of a PxP patch
 *     (spot model versus background only), the appearance model of Sec. V.
 *   - Dynamics are the discrete white-noise-acceleration NCV model.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MODE_RNA 0
#define ORC_MODE_ARNA 1
#define ORC_INIT_TRACKING 0
#define ORC_INIT_INFOSHARE 1
#define ORC_LIK_PATCH 0
#define ORC_LIK_POINT 1
#define ORC_LIK_POISSON 2

/* Philox stream tags (counter word 3, bits 24..31). */
#define TAG_INIT 1u
#define TAG_RING 2u
#define TAG_EXCH 3u
#define TAG_PROP 4u
#define TAG_RESAMPLE 5u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its definition in Salmon, Moraes, Dror and Shaw,      */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC 2011): ten rounds of    */
/* two 32x32->64 multiplications, the Weyl key schedule between rounds.      */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x[1] ^ k0;
        uint32_t y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
        k0 += 0x9E3779B9u; /* golden ratio */
        k1 += 0xBB67AE85u; /* sqrt(3) - 1 */
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* One draw of the project's counter layout: (c0, c1, filter, tag<<24|sub). */
static void draw(uint64_t seed, uint32_t tag, uint32_t sub, uint32_t c0,
                 uint32_t c1, uint32_t f, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, f, (tag << 24) | sub};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* Uniform in (0,1) from the top 23 bits: (2*(r>>9)+1) * 2^-24. */
static double unif24(uint32_t r) { return (2.0 * (double)(r >> 9) + 1.0) / 16777216.0; }
/* Uniform in (0,1) from an 18-bit field b: (2b+1) * 2^-19. */
static double unif18(uint32_t b) { return (2.0 * (double)b + 1.0) / 524288.0; }
/* floor(r * n / 2^32): a bounded integer in [0, n). */
static uint32_t mulshift(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }

/* ------------------------------------------------------------------------ */
/* Step 1 (Alg. 3; Sec. IV-B): random relabelling of the ring.               */
/* Durstenfeld's form of the Fisher-Yates shuffle, i from M-1 down to 1.    */
/* The ring visits pi[0], pi[1], ..., pi[M-1] and closes.  RNA keeps the     */
/* identity labelling, so P_m sends to P_{m+1} and receives from P_{m-1}.   */
/* ------------------------------------------------------------------------ */
void orc_ring(uint64_t seed, uint32_t f, uint32_t k, uint32_t M, int mode,
              uint32_t *pi, uint32_t *pred, uint32_t *succ)
{
    uint32_t *p = (uint32_t *)malloc(sizeof(uint32_t) * (M ? M : 1));
    for (uint32_t i = 0; i < M; ++i) p[i] = i;
    if (mode == ORC_MODE_ARNA) {
        for (uint32_t i = M - 1; i >= 1 && M > 1; --i) {
            uint32_t r[4];
            draw(seed, TAG_RING, 0, i, k, f, r);
            uint32_t j = mulshift(r[0], i + 1);
            uint32_t t = p[i]; p[i] = p[j]; p[j] = t;
        }
    }
    for (uint32_t t = 0; t < M; ++t) {
        uint32_t here = p[t];
        uint32_t nxt = p[(t + 1) % M];
        uint32_t prv = p[(t + M - 1) % M];
        if (pi) pi[t] = here;
        if (succ) succ[here] = nxt;
        if (pred) pred[here] = prv;
    }
    free(p);
}

/* Hardware-aware variant of step 1 (the future work of Sec. VI): the PEs are
 * split into G groups, PE m of filter f in group (f M + m) mod G (on MI355X,
 * with G = 8, the accelerator die its workgroup runs on); the members of each
 * group, in increasing m, are shuffled by Durstenfeld with the draws
 * Philox(i, k, f, RING | 2 + g), the order of the groups by Durstenfeld with
 * Philox(i, k, f, RING | 1); the ring visits the groups in that order, each
 * group's members in their shuffled order, and closes.  Only G of its M edges
 * join different groups.  G <= 1 is the ring of orc_ring. */
void orc_ring_groups(uint64_t seed, uint32_t f, uint32_t k, uint32_t M, uint32_t G,
                     uint32_t *pi, uint32_t *pred, uint32_t *succ)
{
    if (G <= 1 || M <= 1) {
        orc_ring(seed, f, k, M, ORC_MODE_ARNA, pi, pred, succ);
        return;
    }
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * G);
    uint32_t *members = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *p = (uint32_t *)malloc(sizeof(uint32_t) * M);
    for (uint32_t g = 0; g < G; ++g) order[g] = g;
    for (uint32_t i = G - 1; i >= 1; --i) {
        uint32_t r[4];
        draw(seed, TAG_RING, 1, i, k, f, r);
        uint32_t j = mulshift(r[0], i + 1);
        uint32_t t = order[i]; order[i] = order[j]; order[j] = t;
    }
    uint32_t n = 0;
    for (uint32_t a = 0; a < G; ++a) {
        uint32_t g = order[a], cnt = 0;
        for (uint32_t m = 0; m < M; ++m)
            if (((uint64_t)f * M + m) % G == g) members[cnt++] = m;
        for (uint32_t i = cnt - 1; i >= 1 && cnt > 1; --i) {
            uint32_t r[4];
            draw(seed, TAG_RING, 2 + g, i, k, f, r);
            uint32_t j = mulshift(r[0], i + 1);
            uint32_t t = members[i]; members[i] = members[j]; members[j] = t;
        }
        for (uint32_t i = 0; i < cnt; ++i) p[n++] = members[i];
    }
    for (uint32_t t = 0; t < M; ++t) {
        uint32_t here = p[t];
        if (pi) pi[t] = here;
        if (succ) succ[here] = p[(t + 1) % M];
        if (pred) pred[here] = p[(t + M - 1) % M];
    }
    free(order); free(members); free(p);
}

/* ------------------------------------------------------------------------ */
/* Step 2 (Alg. 3; Eq. 3 and Eq. 4): number of particles to exchange.        */
/* P holds the integer PE masses of the previous iteration.                  */
/* ------------------------------------------------------------------------ */
uint32_t orc_fixed_nex(double ratio, uint32_t n_p)
{
    if (!(ratio > 0.0)) return 0;
    if (ratio > 1.0) ratio = 1.0;
    return (uint32_t)floor(ratio * (double)n_p);
}

/* The cut-off as an integer fraction of 10^6; values outside (0, 1) disable it. */
uint32_t orc_cutoff_ppm(double cutoff)
{
    if (!(cutoff > 0.0 && cutoff < 1.0)) return 1000000u;
    return (uint32_t)floor(cutoff * 1e6 + 0.5);
}

uint32_t orc_nex(const uint32_t *P, uint32_t M, uint32_t n_p, int mode,
                 double fixed_ratio, double initial_ratio, double cutoff,
                 int first_iteration)
{
    if (M <= 1) return 0;                                /* one PE: plain SIR */
    if (mode == ORC_MODE_RNA) return orc_fixed_nex(fixed_ratio, n_p);
    if (first_iteration) return orc_fixed_nex(initial_ratio, n_p);
    unsigned __int128 S = 0, D = 0;
    for (uint32_t m = 0; m < M; ++m) {
        S += P[m];
        D += (unsigned __int128)P[m] * P[m];
    }
    if (D == 0) return orc_fixed_nex(0.5, n_p);           /* no mass anywhere */
    /* PE_eff = S^2 / D.  Cut-off: PE_eff > cutoff * M  ->  no exchange. */
    unsigned __int128 S2 = S * S;
    uint32_t ppm = orc_cutoff_ppm(cutoff);
    if ((unsigned __int128)1000000u * S2 > (unsigned __int128)ppm * M * D) return 0;
    /* Eq. 3: N_p [0.5 - 0.5 (S^2/D - 1)/(M-1)] = N_p (M D - S^2) / (2 (M-1) D). */
    unsigned __int128 num = (unsigned __int128)n_p * ((unsigned __int128)M * D - S2);
    unsigned __int128 den = (unsigned __int128)2u * (M - 1) * D;
    return (uint32_t)(num / den);
}

/* Random offset c_m in [0, N_p) of PE m's systematic send selection. */
uint32_t orc_exchange_offset(uint64_t seed, uint32_t f, uint32_t k, uint32_t m, uint32_t n_p)
{
    uint32_t r[4];
    draw(seed, TAG_EXCH, 0, m, k, f, r);
    return mulshift(r[0], n_p);
}

/* The t-th of the N_ex slots PE m sends: floor((t N_p + c_m) / N_ex). */
uint32_t orc_selected_slot(uint32_t t, uint32_t c, uint32_t n_p, uint32_t n_ex)
{
    return (uint32_t)(((uint64_t)t * n_p + c) / n_ex);
}

/* Random offset V_m in [0, T) of PE m's systematic resampling. */
uint32_t orc_resample_offset(uint64_t seed, uint32_t f, uint32_t k, uint32_t m, uint32_t T)
{
    uint32_t r[4];
    draw(seed, TAG_RESAMPLE, 0, m, k, f, r);
    return mulshift(r[0], T);
}

/* ------------------------------------------------------------------------ */
/* Step 7 (Alg. 3; systematic resampling of Alg. 1) on fixed-point weights. */
/* Cumulative sums C_i = Q_0 + ... + Q_i, total T = C_{N_p-1}.  Output j    */
/* takes the first i whose scaled cumulative weight exceeds its pointer:    */
/*     a_j = min { i : N_p C_i > j T + V },   0 <= V < T.                   */
/* Written as the textbook two-index walk over pointers and cumulative sums. */
/* ------------------------------------------------------------------------ */
int orc_resample(const uint32_t *Q, uint32_t n_p, uint32_t V, uint32_t *anc)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (n_p ? n_p : 1));
    uint64_t run = 0;
    for (uint32_t i = 0; i < n_p; ++i) { run += Q[i]; C[i] = run; }
    uint64_t T = run;
    if (n_p == 0) { free(C); return 0; }
    if (T == 0 || (uint64_t)V >= T) { free(C); return -1; }
    uint32_t i = 0;
    for (uint32_t j = 0; j < n_p; ++j) {
        uint64_t pointer = (uint64_t)j * T + V;
        while ((uint64_t)n_p * C[i] <= pointer) ++i;
        anc[j] = i;
    }
    free(C);
    return 0;
}

uint32_t orc_qmax(uint32_t n_p)
{
    uint32_t q = (uint32_t)(0xFFFFFFFFu / (n_p ? n_p : 1));
    return q > (1u << 24) ? (1u << 24) : q;
}

/* ------------------------------------------------------------------------ */
/* Models of the benchmark (Sec. V): state (x, y, vx, vy, I).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t n_filters, n_pe, n_per_pe;
    uint32_t width, height, patch;
    int32_t mode, init_mode, lik_mode;
    double fixed_ratio, initial_ratio, eff_cutoff;
    double psf_sigma, background, noise_sigma;
    double q, sigma_I;
    uint64_t seed;
    uint32_t ring_groups;   /* ARNA: > 1 selects the hardware-aware ring */
} orc_config;

typedef struct { double x, y, vx, vy, I; } particle;

/* The five standard normals of one particle-step from one Philox call.
 * Pairs (r0,r1) and (r2,r3) feed two Box-Muller transforms through their
 * top 23 bits; the low 9 bits of the four words form two 18-bit uniforms for
 * a third transform, of which the cosine branch is used. */
static void five_normals(const uint32_t r[4], double eps[5])
{
    const double two_pi = 6.283185307179586476925286766559;
    double ra = sqrt(-2.0 * log(unif24(r[0]))), ta = two_pi * unif24(r[1]);
    double rb = sqrt(-2.0 * log(unif24(r[2]))), tb = two_pi * unif24(r[3]);
    uint32_t b01 = (r[0] & 511u) | ((r[1] & 511u) << 9);
    uint32_t b23 = (r[2] & 511u) | ((r[3] & 511u) << 9);
    double rc = sqrt(-2.0 * log(unif18(b01))), tc = two_pi * unif18(b23);
    eps[0] = ra * cos(ta);
    eps[1] = ra * sin(ta);
    eps[2] = rb * cos(tb);
    eps[3] = rb * sin(tb);
    eps[4] = rc * cos(tc);
}

/* (P) of Alg. 1: nearly-constant-velocity transition, unit time step.
 * Per axis the noise is N(0, q [[1/3, 1/2], [1/2, 1]]), drawn through the
 * Cholesky factor sqrt(q) [[1/sqrt3, 0], [sqrt3/2, 1/2]]. */
static particle propagate(particle p, const double eps[5], double q, double sigma_I)
{
    double sq = sqrt(q);
    particle n;
    n.x = p.x + p.vx + sq * eps[0] / sqrt(3.0);
    n.vx = p.vx + sq * (sqrt(3.0) / 2.0 * eps[0] + 0.5 * eps[1]);
    n.y = p.y + p.vy + sq * eps[2] / sqrt(3.0);
    n.vy = p.vy + sq * (sqrt(3.0) / 2.0 * eps[2] + 0.5 * eps[3]);
    n.I = p.I + sigma_I * eps[4];
    return n;
}

/* (U) of Alg. 1: log p(z | x) up to an x-independent constant.
 * Patch mode: Gaussian pixel noise, spot = B + I exp(-d^2 / (2 s^2)) over the
 * P x P patch centred on the pixel nearest the particle; the returned value
 * is the log-likelihood ratio against the background-only model,
 *   l = sum_patch [ (z - B)^2 - (z - B - I g)^2 ] / (2 sigma_n^2).
 * Pixels outside the image are skipped.  Pixel (u, v) has its centre at
 * x = u (column), y = v (row).
 * Point mode: z is an observed position, l = -|(x, y) - z|^2 / (2 sigma_n^2).
 * Poisson mode: every pixel is a photon count z ~ Poisson(B + I g) (the noise
 * of the paper's synthetic images, Fig. 1); against the background-only
 * model, log p(z | B + I g) - log p(z | B) = z log(1 + I g / B) - I g.
 *
 * The patch centre is the nearest pixel, floor(x + 1/2) per axis; the sum
 * itself is loglik_at_centre.  A centre more than half a patch outside the
 * image gives l = 0 (no pixel of the patch is in the image). */
static double loglik_at_centre(const orc_config *c, const float *frame, particle p,
                               double fx, double fy)
{
    double s2 = c->noise_sigma * c->noise_sigma;
    int half = (int)c->patch / 2;
    if (!(fx >= -half && fx <= (double)c->width - 1 + half)) return 0.0;
    if (!(fy >= -half && fy <= (double)c->height - 1 + half)) return 0.0;
    long cx = (long)fx, cy = (long)fy;
    double l = 0.0;
    for (long v = cy - half; v <= cy + half; ++v) {
        if (v < 0 || v >= (long)c->height) continue;
        for (long u = cx - half; u <= cx + half; ++u) {
            if (u < 0 || u >= (long)c->width) continue;
            double dx = (double)u - p.x, dy = (double)v - p.y;
            double g = exp(-(dx * dx + dy * dy) / (2.0 * c->psf_sigma * c->psf_sigma));
            double z = (double)frame[(size_t)v * c->width + u];
            if (c->lik_mode == ORC_LIK_POISSON) {
                l += z * log1p(p.I * g / c->background) - p.I * g;
            } else {
                double r0 = z - c->background;
                double r1 = r0 - p.I * g;
                l += (r0 * r0 - r1 * r1) / (2.0 * s2);
            }
        }
    }
    return l;
}

static double log_likelihood(const orc_config *c, const float *frame, uint32_t f, particle p)
{
    if (c->lik_mode == ORC_LIK_POINT) {
        double s2 = c->noise_sigma * c->noise_sigma;
        double dx = p.x - (double)frame[2 * f], dy = p.y - (double)frame[2 * f + 1];
        return -(dx * dx + dy * dy) / (2.0 * s2);
    }
    return loglik_at_centre(c, frame, p, floor(p.x + 0.5), floor(p.y + 0.5));
}

/* The nearest-pixel decision floor(x + 1/2) of a coordinate computed with a
 * rounding error of at most eps may land on either side of a pixel boundary
 * (x + 1/2 an integer) when x lies within eps of it: both centres are then
 * valid outcomes of the decision.  Returns 1 and the other centre in *alt
 * when that is the case. */
static int centre_ambiguous(double x, double eps_rel, double eps_abs, double *alt)
{
    double t = x + 0.5, b = floor(t + 0.5);
    double eps = eps_rel * (fabs(x) > 1.0 ? fabs(x) : 1.0) + eps_abs;
    if (!(fabs(t - b) <= eps)) return 0;
    double c0 = floor(t);
    *alt = (c0 == b) ? b - 1.0 : b;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* The filter object: particles, per-PE log weights, iteration counter.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_config cfg;
    uint32_t k;           /* completed iterations */
    particle *s;          /* [N] resampled particles of iteration k */
    double *L;            /* [F*M] log W^(m)_k (0 before the first iteration) */
    int *lineage;         /* [N] optional tag: PE a particle's lineage started on */
    double amb_rel, amb_abs;  /* > 0: record the alternative patch centres (see
                                 orc_set_ambiguity) */
} orc_filter;

/* Per-iteration outputs; every pointer may be NULL. */
typedef struct {
    uint32_t *ring_pi;    /* [F][M] ring order */
    uint32_t *ring_pred;  /* [F][M] */
    uint32_t *n_ex;       /* [F] */
    uint32_t *exch_off;   /* [F][M] c_m */
    int64_t *src_map;     /* [N] slot g <- slot src_map[g] */
    double *lambda;       /* [N] carried log weight after renormalization */
    double *prop;         /* [5][N] propagated particles */
    double *ell;          /* [N] log-likelihood */
    uint32_t *Q;          /* [N] fixed-point weights */
    uint32_t *T;          /* [F][M] */
    uint32_t *V;          /* [F][M] */
    uint32_t *anc;        /* [N] ancestor slot within the PE */
    double *state;        /* [5][N] resampled particles */
    double *L_pe;         /* [F][M] log W^(m)_k */
    double *lstar;        /* [F][M] max of lambda + ell */
    double *xhat_pe;      /* [F][M][5] */
    double *xhat;         /* [F][5] */
    double *L_glob;       /* [F] log W_k */
    uint32_t *P;          /* [F][M] integer PE masses */
    double *pe_eff;       /* [F] */
    double *log_z;        /* [F] log p(z_k | z_1:k-1) (ratio form) */
    uint32_t *n_ex_next;  /* [F] what step 2 of the next iteration will use */
    int32_t *lineage;     /* [N] lineage tag after resampling */
    uint32_t *amb;        /* [N] bit 0 / bit 1: the x / y patch centre is ambiguous */
    double *ell_alt;      /* [N][3] l with the other x centre, other y centre, both
                             (NaN where that alternative does not exist) */
} orc_trace;

static size_t n_total(const orc_config *c) { return (size_t)c->n_filters * c->n_pe * c->n_per_pe; }

void orc_destroy(orc_filter *o)
{
    if (!o) return;
    free(o->s); free(o->L); free(o->lineage); free(o);
}

/* Initialization of the two benchmark modes (Sec. V).
 * Tracking: every particle at the true state.
 * Information sharing: PE 0 near the truth (uniform in the radius-2 disk,
 * true velocity and intensity); the other PEs uniform over the image,
 * velocity uniform in [-2, 2]^2, intensity uniform in [0, 2 I_true]. */
orc_filter *orc_create(const orc_config *cfg, const double *truth /* [F][5] */)
{
    if (!cfg || cfg->n_filters == 0 || cfg->n_pe == 0 || cfg->n_per_pe == 0) return NULL;
    orc_filter *o = (orc_filter *)calloc(1, sizeof(orc_filter));
    o->cfg = *cfg;
    size_t N = n_total(cfg);
    o->s = (particle *)malloc(sizeof(particle) * N);
    o->L = (double *)calloc((size_t)cfg->n_filters * cfg->n_pe, sizeof(double));
    o->lineage = (int *)malloc(sizeof(int) * N);
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t M = cfg->n_pe, np = cfg->n_per_pe;
    for (uint32_t f = 0; f < cfg->n_filters; ++f) {
        const double *t = truth + 5 * f;
        for (uint32_t m = 0; m < M; ++m) {
            for (uint32_t s = 0; s < np; ++s) {
                size_t g = ((size_t)f * M + m) * np + s;
                uint32_t j = m * np + s;
                particle p = {t[0], t[1], t[2], t[3], t[4]};
                if (cfg->init_mode == ORC_INIT_INFOSHARE) {
                    uint32_t r0[4], r1[4];
                    draw(cfg->seed, TAG_INIT, 0, j, 0, f, r0);
                    draw(cfg->seed, TAG_INIT, 1, j, 0, f, r1);
                    if (m == 0) {
                        double rad = 2.0 * sqrt(unif24(r0[0]));
                        double ang = two_pi * unif24(r0[1]);
                        p.x = t[0] + rad * cos(ang);
                        p.y = t[1] + rad * sin(ang);
                    } else {
                        p.x = -0.5 + (double)cfg->width * unif24(r0[0]);
                        p.y = -0.5 + (double)cfg->height * unif24(r0[1]);
                        p.vx = -2.0 + 4.0 * unif24(r0[2]);
                        p.vy = -2.0 + 4.0 * unif24(r0[3]);
                        p.I = 2.0 * t[4] * unif24(r1[0]);
                    }
                }
                o->s[g] = p;
                o->lineage[g] = (int)m;
            }
        }
    }
    return o;
}

/* Replace particles ([5][N] component-major), log weights ([F][M]) and the
 * count of completed iterations.  L may be NULL (all zero). */
int orc_set_state(orc_filter *o, const double *state, const double *L, uint32_t k)
{
    size_t N = n_total(&o->cfg);
    for (size_t g = 0; g < N; ++g) {
        o->s[g].x = state[0 * N + g];
        o->s[g].y = state[1 * N + g];
        o->s[g].vx = state[2 * N + g];
        o->s[g].vy = state[3 * N + g];
        o->s[g].I = state[4 * N + g];
    }
    size_t FM = (size_t)o->cfg.n_filters * o->cfg.n_pe;
    for (size_t i = 0; i < FM; ++i) o->L[i] = L ? L[i] : 0.0;
    o->k = k;
    return 0;
}

int orc_get_state(const orc_filter *o, double *state, double *L, uint32_t *k)
{
    size_t N = n_total(&o->cfg);
    if (state)
        for (size_t g = 0; g < N; ++g) {
            state[0 * N + g] = o->s[g].x;
            state[1 * N + g] = o->s[g].y;
            state[2 * N + g] = o->s[g].vx;
            state[3 * N + g] = o->s[g].vy;
            state[4 * N + g] = o->s[g].I;
        }
    size_t FM = (size_t)o->cfg.n_filters * o->cfg.n_pe;
    if (L) for (size_t i = 0; i < FM; ++i) L[i] = o->L[i];
    if (k) *k = o->k;
    return 0;
}

int orc_set_lineage(orc_filter *o, const int32_t *tag)
{
    size_t N = n_total(&o->cfg);
    for (size_t g = 0; g < N; ++g) o->lineage[g] = tag[g];
    return 0;
}

static double logsumexp(const double *a, size_t n)
{
    double mx = -INFINITY;
    for (size_t i = 0; i < n; ++i) if (a[i] > mx) mx = a[i];
    if (mx == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += exp(a[i] - mx);
    return mx + log(s);
}

/* Integer PE masses of the master step: P_m = floor(exp(L_m - max L) 2^20). */
static void pe_masses(const double *L, uint32_t M, uint32_t *P)
{
    double mx = -INFINITY;
    for (uint32_t m = 0; m < M; ++m) if (L[m] > mx) mx = L[m];
    for (uint32_t m = 0; m < M; ++m)
        P[m] = (mx == -INFINITY) ? 0u : (uint32_t)floor(exp(L[m] - mx) * 1048576.0);
}

/* Steps 6-7 of Alg. 3 for one PE (filter f, PE m, iteration k): from the
 * carried log-weights lam[i] (step 4) and log-likelihoods ell[i] (step 5) of
 * its n_p particles prop[i], the local estimate x^m (6), the log weight sum
 * L = log W^(m) and its maximum term lstar, and local systematic resampling
 * (7) on the fixed-point weights Q_i = floor(w_i Q_max), w_i = e^{lam+ell-lstar}:
 * total T, offset V and ancestors anc[j].  Returns 0, or -4 when the weights
 * are unusable (NaN, or all zero): the ancestors are then the identity. */
int orc_pe_update(const orc_config *c, uint32_t f, uint32_t k, uint32_t m, uint32_t np,
                  const double *lam, const double *ell, const double *prop /* [5][np] */,
                  double xm[5], double *L_out, double *lstar_out, uint32_t *Q, uint32_t *T_out,
                  uint32_t *V_out, uint32_t *anc)
{
    int status = 0;
    const uint32_t qmax = orc_qmax(np);
    /* 6: local estimate and local weight sum, with the max subtracted. */
    double lstar = -INFINITY;
    for (uint32_t s = 0; s < np; ++s) {
        double u = lam[s] + ell[s];
        if (u > lstar) lstar = u;
    }
    double *w = (double *)malloc(sizeof(double) * np);
    double wsum = 0.0;
    for (uint32_t s = 0; s < np; ++s) {
        w[s] = (lstar == -INFINITY) ? 1.0 : exp(lam[s] + ell[s] - lstar);
        wsum += w[s];
    }
    for (int d = 0; d < 5; ++d) {
        double acc = 0.0;
        for (uint32_t s = 0; s < np; ++s) acc += w[s] * prop[(size_t)d * np + s];
        xm[d] = acc / wsum;
    }
    *L_out = (lstar == -INFINITY) ? -INFINITY : lstar + log(wsum);
    *lstar_out = lstar;

    /* 7: systematic resampling with the locally normalized weights,
     * represented as Q_i = floor(w_i Q_max). */
    uint64_t T = 0;
    for (uint32_t s = 0; s < np; ++s) {
        double qd = floor(w[s] * (double)qmax);
        if (!(qd >= 0.0)) qd = 0.0;          /* NaN guard */
        if (qd > (double)qmax) qd = (double)qmax;
        Q[s] = (uint32_t)qd;
        T += Q[s];
    }
    uint32_t V = 0;
    if (T > 0 && T <= 0xFFFFFFFFull) {
        V = orc_resample_offset(c->seed, f, k, m, (uint32_t)T);
        orc_resample(Q, np, V, anc);
    } else {
        for (uint32_t s = 0; s < np; ++s) anc[s] = s;
        status = -4;
    }
    for (uint32_t s = 0; s < np; ++s)
        if (isnan(ell[s])) status = -4;
    *T_out = (uint32_t)T;
    *V_out = V;
    free(w);
    return status;
}

/* Steps 9-10 of Alg. 3 for one filter: from the M PE log masses L[m] =
 * log W^(m)_k and estimates xm[m][5], the master's W_k (as L_glob), the
 * global estimate x_k = sum_m W^(m) x^m / W_k, the integer PE masses
 * P_m = floor(e^{L_m - max L} 2^20) behind Eq. 4, PE_eff = S^2 / D, the
 * likelihood increment log p(z_k | z_1..z_{k-1}) = L_glob - log N_p (the
 * carried weights of the step sum to N_p), and the N_ex of Eq. 3 for the
 * next iteration.  Every output pointer may be NULL. */
void orc_master(const orc_config *c, const double *L, const double *xm, double *L_glob,
                double xhat[5], uint32_t *P_out, double *pe_eff, double *log_z,
                uint32_t *nex_next)
{
    const uint32_t M = c->n_pe, np = c->n_per_pe;
    double Lg = logsumexp(L, M);
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * M);
    pe_masses(L, M, P);
    double S = 0.0, D = 0.0;
    for (uint32_t m = 0; m < M; ++m) { S += (double)P[m]; D += (double)P[m] * (double)P[m]; }
    double acc[5] = {0, 0, 0, 0, 0};
    for (uint32_t m = 0; m < M; ++m) {
        if (L[m] == -INFINITY) continue;
        double wm = exp(L[m] - Lg);
        for (int d = 0; d < 5; ++d) acc[d] += wm * xm[(size_t)m * 5 + d];
    }
    if (L_glob) *L_glob = Lg;
    if (P_out) memcpy(P_out, P, sizeof(uint32_t) * M);
    if (pe_eff) *pe_eff = D > 0 ? S * S / D : 0.0;
    if (log_z) *log_z = Lg - log((double)np);
    if (nex_next)
        *nex_next = orc_nex(P, M, np, c->mode, c->fixed_ratio, c->initial_ratio, c->eff_cutoff, 0);
    if (xhat) for (int d = 0; d < 5; ++d) xhat[d] = acc[d];
    free(P);
}

/* Record, from the next orc_step on, which patch centres are ambiguous for a
 * coordinate error of eps_rel * max(|x|, 1) + eps_abs, and the likelihoods at
 * the other centres (trace fields amb, ell_alt).  Zero turns it off. */
void orc_set_ambiguity(orc_filter *o, double eps_rel, double eps_abs)
{
    o->amb_rel = eps_rel;
    o->amb_abs = eps_abs;
}

/* One iteration k = o->k + 1 of Alg. 3 (ARNA) or Alg. 2 (RNA) on every filter.
 * frame: patch mode [H][W] row-major; point mode [F][2]. */
int orc_step(orc_filter *o, const float *frame, orc_trace *tr)
{
    const orc_config *c = &o->cfg;
    const uint32_t F = c->n_filters, M = c->n_pe, np = c->n_per_pe;
    const size_t N = n_total(c);
    const uint32_t k = o->k + 1;
    int status = 0;

    particle *src_particles = (particle *)malloc(sizeof(particle) * N);
    int *src_lineage = (int *)malloc(sizeof(int) * N);
    double *lam = (double *)malloc(sizeof(double) * N);
    particle *prop = (particle *)malloc(sizeof(particle) * N);
    double *ell = (double *)malloc(sizeof(double) * N);
    double *Lnew = (double *)malloc(sizeof(double) * F * M);
    double *xm_all = (double *)malloc(sizeof(double) * F * M * 5);
    uint32_t *pred = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *pi = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *coff = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *Pprev = (uint32_t *)malloc(sizeof(uint32_t) * M);

    for (uint32_t f = 0; f < F; ++f) {
        const double *Lprev = o->L + (size_t)f * M;

        /* 1: ring for this iteration. */
        if (c->mode == ORC_MODE_ARNA && c->ring_groups > 1)
            orc_ring_groups(c->seed, f, k, M, c->ring_groups, pi, pred, NULL);
        else
            orc_ring(c->seed, f, k, M, c->mode, pi, pred, NULL);

        /* 2: exchange ratio from the previous iteration's PE masses. */
        pe_masses(Lprev, M, Pprev);
        uint32_t nex = orc_nex(Pprev, M, np, c->mode, c->fixed_ratio, c->initial_ratio,
                               c->eff_cutoff, o->k == 0);
        if (tr && tr->n_ex) tr->n_ex[f] = nex;
        if (tr && tr->ring_pi) memcpy(tr->ring_pi + (size_t)f * M, pi, sizeof(uint32_t) * M);
        if (tr && tr->ring_pred) memcpy(tr->ring_pred + (size_t)f * M, pred, sizeof(uint32_t) * M);

        /* 3: exchange.  Every slot first keeps its own particle; then PE m's
         * selected slots are refilled with the particles that pred(m) sends,
         * which are pred(m)'s own selected slots. */
        for (uint32_t m = 0; m < M; ++m) coff[m] = orc_exchange_offset(c->seed, f, k, m, np);
        if (tr && tr->exch_off) memcpy(tr->exch_off + (size_t)f * M, coff, sizeof(uint32_t) * M);
        size_t base = (size_t)f * M * np;
        int64_t *origin_pe = (int64_t *)malloc(sizeof(int64_t) * (size_t)M * np);
        for (uint32_t m = 0; m < M; ++m)
            for (uint32_t s = 0; s < np; ++s) {
                size_t g = base + (size_t)m * np + s;
                src_particles[g] = o->s[g];
                src_lineage[g] = o->lineage[g];
                origin_pe[(size_t)m * np + s] = m;
                if (tr && tr->src_map) tr->src_map[g] = (int64_t)g;
            }
        if (M > 1 && nex > 0) {
            for (uint32_t m = 0; m < M; ++m) {
                uint32_t from = pred[m];
                for (uint32_t t = 0; t < nex; ++t) {
                    uint32_t dst_slot = orc_selected_slot(t, coff[m], np, nex);
                    uint32_t src_slot = orc_selected_slot(t, coff[from], np, nex);
                    size_t g = base + (size_t)m * np + dst_slot;
                    size_t gs = base + (size_t)from * np + src_slot;
                    src_particles[g] = o->s[gs];
                    src_lineage[g] = o->lineage[gs];
                    origin_pe[(size_t)m * np + dst_slot] = from;
                    if (tr && tr->src_map) tr->src_map[g] = (int64_t)gs;
                }
            }
        }

        /* 4: renormalize the carried weights by W_{k-1} = sum_m W^(m)_{k-1}. */
        double Lglob_prev = logsumexp(Lprev, M);
        for (size_t i = 0; i < (size_t)M * np; ++i)
            lam[base + i] = Lprev[origin_pe[i]] - Lglob_prev;
        free(origin_pe);
    }

    /* 5-8 on every PE independently. */
    const int amb_on = (o->amb_rel > 0.0 || o->amb_abs > 0.0) && c->lik_mode != ORC_LIK_POINT;
    #pragma omp parallel for schedule(static)
    for (long fm = 0; fm < (long)F * M; ++fm) {
        uint32_t f = (uint32_t)(fm / M), m = (uint32_t)(fm % M);
        size_t base = (size_t)fm * np;

        /* 5: (P) and (U). */
        for (uint32_t s = 0; s < np; ++s) {
            size_t g = base + s;
            uint32_t r[4];
            draw(c->seed, TAG_PROP, 0, m * np + s, k, f, r);
            double eps[5];
            five_normals(r, eps);
            prop[g] = propagate(src_particles[g], eps, c->q, c->sigma_I);
            ell[g] = log_likelihood(c, frame, f, prop[g]);
            if (amb_on && tr && (tr->amb || tr->ell_alt)) {
                const particle p = prop[g];
                double ax = 0.0, ay = 0.0;
                uint32_t bits = (uint32_t)centre_ambiguous(p.x, o->amb_rel, o->amb_abs, &ax) |
                                ((uint32_t)centre_ambiguous(p.y, o->amb_rel, o->amb_abs, &ay) << 1);
                if (tr->amb) tr->amb[g] = bits;
                if (tr->ell_alt) {
                    const double fx = floor(p.x + 0.5), fy = floor(p.y + 0.5);
                    tr->ell_alt[3 * g + 0] = (bits & 1u) ? loglik_at_centre(c, frame, p, ax, fy) : NAN;
                    tr->ell_alt[3 * g + 1] = (bits & 2u) ? loglik_at_centre(c, frame, p, fx, ay) : NAN;
                    tr->ell_alt[3 * g + 2] = (bits == 3u) ? loglik_at_centre(c, frame, p, ax, ay) : NAN;
                }
            }
        }

        /* 6-7: local estimate, weight sum and systematic resampling. */
        double *pc = (double *)malloc(sizeof(double) * 5 * np);
        for (uint32_t s = 0; s < np; ++s) {
            const particle *p = &prop[base + s];
            pc[0 * (size_t)np + s] = p->x; pc[1 * (size_t)np + s] = p->y;
            pc[2 * (size_t)np + s] = p->vx; pc[3 * (size_t)np + s] = p->vy;
            pc[4 * (size_t)np + s] = p->I;
        }
        uint32_t *Q = (uint32_t *)malloc(sizeof(uint32_t) * np);
        uint32_t *anc = (uint32_t *)malloc(sizeof(uint32_t) * np);
        double xm[5], Lm, lstar;
        uint32_t T, V;
        int st = orc_pe_update(c, f, k, m, np, lam + base, ell + base, pc, xm, &Lm, &lstar, Q, &T,
                               &V, anc);
        if (st != 0) {
            #pragma omp atomic write
            status = st;
        }
        for (int d = 0; d < 5; ++d) xm_all[(size_t)fm * 5 + d] = xm[d];
        /* 8: every resampled particle of PE m carries W^(m)_k. */
        for (uint32_t j = 0; j < np; ++j) {
            o->s[base + j] = prop[base + anc[j]];
            o->lineage[base + j] = src_lineage[base + anc[j]];
        }
        Lnew[fm] = Lm;

        if (tr) {
            if (tr->Q) memcpy(tr->Q + base, Q, sizeof(uint32_t) * np);
            if (tr->anc) memcpy(tr->anc + base, anc, sizeof(uint32_t) * np);
            if (tr->T) tr->T[fm] = T;
            if (tr->V) tr->V[fm] = V;
            if (tr->L_pe) tr->L_pe[fm] = Lm;
            if (tr->lstar) tr->lstar[fm] = lstar;
            if (tr->xhat_pe) for (int d = 0; d < 5; ++d) tr->xhat_pe[fm * 5 + d] = xm[d];
        }
        free(Q); free(anc); free(pc);
    }

    /* 9-10: master: W_k = sum_m W^(m)_k, the global estimate
     * x_k = sum_m W^(m)_k x^m_k / W_k, and the PE masses behind Eq. 4. */
    for (uint32_t f = 0; f < F; ++f) {
        if (!tr) continue;
        orc_master(c, Lnew + (size_t)f * M, xm_all + (size_t)f * M * 5,
                   tr->L_glob ? tr->L_glob + f : NULL, tr->xhat ? tr->xhat + 5 * f : NULL,
                   tr->P ? tr->P + (size_t)f * M : NULL, tr->pe_eff ? tr->pe_eff + f : NULL,
                   tr->log_z ? tr->log_z + f : NULL, tr->n_ex_next ? tr->n_ex_next + f : NULL);
    }

    if (tr) {
        if (tr->lambda) memcpy(tr->lambda, lam, sizeof(double) * N);
        if (tr->ell) memcpy(tr->ell, ell, sizeof(double) * N);
        if (tr->prop)
            for (size_t g = 0; g < N; ++g) {
                tr->prop[0 * N + g] = prop[g].x; tr->prop[1 * N + g] = prop[g].y;
                tr->prop[2 * N + g] = prop[g].vx; tr->prop[3 * N + g] = prop[g].vy;
                tr->prop[4 * N + g] = prop[g].I;
            }
        if (tr->state)
            for (size_t g = 0; g < N; ++g) {
                tr->state[0 * N + g] = o->s[g].x; tr->state[1 * N + g] = o->s[g].y;
                tr->state[2 * N + g] = o->s[g].vx; tr->state[3 * N + g] = o->s[g].vy;
                tr->state[4 * N + g] = o->s[g].I;
            }
        if (tr->lineage) for (size_t g = 0; g < N; ++g) tr->lineage[g] = o->lineage[g];
    }

    memcpy(o->L, Lnew, sizeof(double) * F * M);
    o->k = k;
    free(src_particles); free(src_lineage); free(lam); free(prop); free(ell); free(Lnew); free(xm_all);
    free(pred); free(pi); free(coff); free(Pprev);
    return status;
}

/* Sets the OpenMP thread count of later calls (no effect without OpenMP). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Threads the OpenMP runtime will use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Single-particle entry points used by the oracle's own pin tests.          */
/* ------------------------------------------------------------------------ */
void orc_normals(uint64_t seed, uint32_t f, uint32_t k, uint32_t j, double eps[5])
{
    uint32_t r[4];
    draw(seed, TAG_PROP, 0, j, k, f, r);
    five_normals(r, eps);
}

void orc_propagate(const double in[5], const double eps[5], double q, double sigma_I, double out[5])
{
    particle p = {in[0], in[1], in[2], in[3], in[4]};
    particle n = propagate(p, eps, q, sigma_I);
    out[0] = n.x; out[1] = n.y; out[2] = n.vx; out[3] = n.vy; out[4] = n.I;
}

double orc_loglik(const orc_config *c, const float *frame, uint32_t f, const double st[5])
{
    particle p = {st[0], st[1], st[2], st[3], st[4]};
    return log_likelihood(c, frame, f, p);
}

/* ------------------------------------------------------------------------ */
/* Gradient of the log marginal likelihood with the discrete choices frozen */
/* ------------------------------------------------------------------------ */
/* For a run of K iterations the filter's estimate of log p(z_1..z_K) is, per
 * filter, J = sum_k (log W_k - log N_p), W_k = sum_m W^(m)_k of step 9 (the
 * carried weights are renormalized by W_{k-1} in step 4, so the increments
 * chain).  Hold every discrete choice of the run fixed -- ring, N_ex, the
 * exchanged slots, the ancestors of step 7 and the patch centres of the
 * likelihood -- and the normals fixed by their Philox counters; J is then a
 * smooth function of theta = (psf_sigma, I0, q), where I0 shifts the
 * intensity of every particle of the starting state.
 *
 * orc_grad runs K iterations exactly as orc_step does (so its choices are
 * the filter's own) and carries alongside every particle its derivative
 * d(particle)/d(theta), and alongside every PE d(log W^(m))/d(theta): forward
 * differentiation of each step by the chain rule.  It can record the choices
 * (a tape); orc_replay evaluates J at another theta with those choices, which
 * is what finite differences of the frozen objective need.
 *
 * Both run from the filter's start (orc_create) over K frames stored one
 * after another.  Patch likelihood only. */

#define NTH 3   /* theta = (psf_sigma, I0, q) */

typedef struct {
    particle p;
    double d[5][NTH];   /* d(x, y, vx, vy, I) / d(theta) */
} dual_particle;

/* Patch log-likelihood with a fixed centre (cx, cy) and its partial
 * derivatives in x, y, I and psf_sigma.  The value is computed exactly as
 * log_likelihood does; per pixel, with r0 = z - B and g the PSF,
 *   l_pix = (r0^2 - (r0 - I g)^2) / (2 s_n^2),
 *   dl_pix/dg = I (r0 - I g) / s_n^2,   dl_pix/dI = g (r0 - I g) / s_n^2,
 *   dg/dx = g (u - x) / s^2,  dg/dy = g (v - y) / s^2,
 *   dg/ds = g ((u - x)^2 + (v - y)^2) / s^3. */
static double loglik_centred(const orc_config *c, double psf_sigma, const float *frame,
                             long cx, long cy, particle p, double grad[4])
{
    double s2 = c->noise_sigma * c->noise_sigma;
    double ps2 = psf_sigma * psf_sigma;
    int half = (int)c->patch / 2;
    double l = 0.0;
    grad[0] = grad[1] = grad[2] = grad[3] = 0.0;
    for (long v = cy - half; v <= cy + half; ++v) {
        if (v < 0 || v >= (long)c->height) continue;
        for (long u = cx - half; u <= cx + half; ++u) {
            if (u < 0 || u >= (long)c->width) continue;
            double dx = (double)u - p.x, dy = (double)v - p.y;
            double g = exp(-(dx * dx + dy * dy) / (2.0 * ps2));
            double z = (double)frame[(size_t)v * c->width + u];
            double r0 = z - c->background;
            double r1 = r0 - p.I * g;
            l += (r0 * r0 - r1 * r1) / (2.0 * s2);
            double dl_dg = p.I * r1 / s2;
            grad[0] += dl_dg * g * dx / ps2;
            grad[1] += dl_dg * g * dy / ps2;
            grad[2] += g * r1 / s2;
            grad[3] += dl_dg * g * (dx * dx + dy * dy) / (ps2 * psf_sigma);
        }
    }
    return l;
}

/* The patch centre of log_likelihood, or 0 when the patch misses the image. */
static int patch_centre(const orc_config *c, particle p, int32_t *cx, int32_t *cy)
{
    int half = (int)c->patch / 2;
    double fx = floor(p.x + 0.5), fy = floor(p.y + 0.5);
    if (!(fx >= -half && fx <= (double)c->width - 1 + half)) return 0;
    if (!(fy >= -half && fy <= (double)c->height - 1 + half)) return 0;
    *cx = (int32_t)fx;
    *cy = (int32_t)fy;
    return 1;
}

/* One run.  record != 0: choices computed as in orc_step and written to the
 * tape (each tape pointer may be NULL); record == 0: choices read from the
 * tape.  dJ (nullable) receives dJ/dtheta. */
static int run_frozen(const orc_config *cfg, const double *truth, double dI0,
                      const float *frames, uint32_t K, int record,
                      uint32_t *tape_nex, uint32_t *tape_anc, int32_t *tape_centre,
                      double *J, double *dJ)
{
    if (cfg->lik_mode != ORC_LIK_PATCH) return -6;
    const uint32_t F = cfg->n_filters, M = cfg->n_pe, np = cfg->n_per_pe;
    const size_t N = n_total(cfg), frame_size = (size_t)cfg->width * cfg->height;
    const uint32_t qmax = orc_qmax(np);
    const double sq = sqrt(cfg->q), dsq = 0.5 / sq;   /* sqrt(q) and its q-derivative */
    int status = 0;

    orc_filter *o = orc_create(cfg, truth);
    if (!o) return -1;
    dual_particle *s = (dual_particle *)calloc(N, sizeof(dual_particle));
    dual_particle *src = (dual_particle *)malloc(sizeof(dual_particle) * N);
    dual_particle *prop = (dual_particle *)malloc(sizeof(dual_particle) * N);
    double *lam = (double *)malloc(sizeof(double) * N);
    double *dlam = (double *)malloc(sizeof(double) * N * NTH);
    double *ell = (double *)malloc(sizeof(double) * N);
    double *dell = (double *)malloc(sizeof(double) * N * NTH);
    double *L = (double *)calloc((size_t)F * M, sizeof(double));
    double *dL = (double *)calloc((size_t)F * M * NTH, sizeof(double));
    double *Lnew = (double *)malloc(sizeof(double) * F * M);
    double *dLnew = (double *)malloc(sizeof(double) * F * M * NTH);
    uint32_t *pred = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *pi = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *coff = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * M);
    uint32_t *origin_pe = (uint32_t *)malloc(sizeof(uint32_t) * N);
    for (size_t g = 0; g < N; ++g) {
        s[g].p = o->s[g];
        s[g].p.I += dI0;
        s[g].d[4][1] = 1.0;          /* dI/dI0 */
    }
    for (uint32_t f = 0; f < F; ++f) {
        J[f] = 0.0;
        if (dJ) for (int j = 0; j < NTH; ++j) dJ[f * NTH + j] = 0.0;
    }

    for (uint32_t k = 1; k <= K; ++k) {
        const float *frame = frames + (size_t)(k - 1) * frame_size;
        /* steps 1-4: ring, N_ex, exchange, renormalized carried weights */
        for (uint32_t f = 0; f < F; ++f) {
            const double *Lf = L + (size_t)f * M;
            const double *dLf = dL + (size_t)f * M * NTH;
            if (cfg->mode == ORC_MODE_ARNA && cfg->ring_groups > 1)
                orc_ring_groups(cfg->seed, f, k, M, cfg->ring_groups, pi, pred, NULL);
            else
                orc_ring(cfg->seed, f, k, M, cfg->mode, pi, pred, NULL);
            uint32_t nex;
            if (record) {
                pe_masses(Lf, M, P);
                nex = orc_nex(P, M, np, cfg->mode, cfg->fixed_ratio, cfg->initial_ratio,
                              cfg->eff_cutoff, k == 1);
                if (tape_nex) tape_nex[(size_t)(k - 1) * F + f] = nex;
            } else {
                nex = tape_nex[(size_t)(k - 1) * F + f];
            }
            for (uint32_t m = 0; m < M; ++m) coff[m] = orc_exchange_offset(cfg->seed, f, k, m, np);
            size_t base = (size_t)f * M * np;
            for (uint32_t m = 0; m < M; ++m)
                for (uint32_t t = 0; t < np; ++t) {
                    src[base + (size_t)m * np + t] = s[base + (size_t)m * np + t];
                    origin_pe[base + (size_t)m * np + t] = m;
                }
            if (M > 1 && nex > 0)
                for (uint32_t m = 0; m < M; ++m)
                    for (uint32_t t = 0; t < nex; ++t) {
                        size_t g = base + (size_t)m * np + orc_selected_slot(t, coff[m], np, nex);
                        size_t gs = base + (size_t)pred[m] * np +
                                    orc_selected_slot(t, coff[pred[m]], np, nex);
                        src[g] = s[gs];
                        origin_pe[g] = pred[m];
                    }
            /* lambda = L_origin - log sum_m W_m; its derivative subtracts the
             * mass-weighted mean of dL */
            double Lg = logsumexp(Lf, M);
            double mean_dL[NTH] = {0, 0, 0};
            for (uint32_t m = 0; m < M; ++m) {
                double pm = (Lg == -INFINITY) ? 0.0 : exp(Lf[m] - Lg);
                for (int j = 0; j < NTH; ++j) mean_dL[j] += pm * dLf[m * NTH + j];
            }
            for (size_t i = base; i < base + (size_t)M * np; ++i) {
                lam[i] = Lf[origin_pe[i]] - Lg;
                for (int j = 0; j < NTH; ++j)
                    dlam[i * NTH + j] = dLf[origin_pe[i] * NTH + j] - mean_dL[j];
            }
        }

        /* steps 5-8 per PE */
        #pragma omp parallel for schedule(static)
        for (long fm = 0; fm < (long)F * M; ++fm) {
            uint32_t f = (uint32_t)(fm / M), m = (uint32_t)(fm % M);
            size_t base = (size_t)fm * np;
            for (uint32_t t = 0; t < np; ++t) {
                size_t g = base + t;
                uint32_t r[4];
                double eps[5];
                draw(cfg->seed, TAG_PROP, 0, m * np + t, k, f, r);
                five_normals(r, eps);
                dual_particle *a = &src[g], *b = &prop[g];
                b->p = propagate(a->p, eps, cfg->q, cfg->sigma_I);
                /* tangent of the NCV step: position += velocity, and the
                 * noise scales with sqrt(q) */
                for (int j = 0; j < NTH; ++j) {
                    double nq = (j == 2) ? dsq : 0.0;
                    b->d[0][j] = a->d[0][j] + a->d[2][j] + nq * eps[0] / sqrt(3.0);
                    b->d[2][j] = a->d[2][j] + nq * (sqrt(3.0) / 2.0 * eps[0] + 0.5 * eps[1]);
                    b->d[1][j] = a->d[1][j] + a->d[3][j] + nq * eps[2] / sqrt(3.0);
                    b->d[3][j] = a->d[3][j] + nq * (sqrt(3.0) / 2.0 * eps[2] + 0.5 * eps[3]);
                    b->d[4][j] = a->d[4][j];
                }
                int32_t cx = 0, cy = 0;
                int has;
                int32_t *tc = tape_centre ? tape_centre + ((size_t)(k - 1) * N + g) * 2 : NULL;
                if (record) {
                    has = patch_centre(cfg, b->p, &cx, &cy);
                    if (tc) { tc[0] = has ? cx : INT32_MIN; tc[1] = has ? cy : INT32_MIN; }
                } else {
                    has = tc[0] != INT32_MIN;
                    cx = tc[0];
                    cy = tc[1];
                }
                double gr[4] = {0, 0, 0, 0};
                ell[g] = has ? loglik_centred(cfg, cfg->psf_sigma, frame, cx, cy, b->p, gr) : 0.0;
                for (int j = 0; j < NTH; ++j)
                    dell[g * NTH + j] = gr[0] * b->d[0][j] + gr[1] * b->d[1][j] +
                                        gr[2] * b->d[4][j] + (j == 0 ? gr[3] : 0.0);
            }
            /* step 6 and the derivative of log W^(m) = log sum exp(u) */
            double lstar = -INFINITY;
            for (uint32_t t = 0; t < np; ++t) {
                double u = lam[base + t] + ell[base + t];
                if (u > lstar) lstar = u;
            }
            double *w = (double *)malloc(sizeof(double) * np);
            double wsum = 0.0, dsum[NTH] = {0, 0, 0};
            for (uint32_t t = 0; t < np; ++t) {
                w[t] = (lstar == -INFINITY) ? 1.0 : exp(lam[base + t] + ell[base + t] - lstar);
                wsum += w[t];
                for (int j = 0; j < NTH; ++j)
                    dsum[j] += w[t] * (dlam[(base + t) * NTH + j] + dell[(base + t) * NTH + j]);
            }
            Lnew[fm] = (lstar == -INFINITY) ? -INFINITY : lstar + log(wsum);
            for (int j = 0; j < NTH; ++j) dLnew[fm * NTH + j] = dsum[j] / wsum;
            /* step 7: ancestors (computed as in orc_step, or from the tape) */
            uint32_t *anc = (uint32_t *)malloc(sizeof(uint32_t) * np);
            uint32_t *ta = tape_anc ? tape_anc + (size_t)(k - 1) * N + base : NULL;
            if (record) {
                uint32_t *Q = (uint32_t *)malloc(sizeof(uint32_t) * np);
                uint64_t T = 0;
                for (uint32_t t = 0; t < np; ++t) {
                    double qd = floor(w[t] * (double)qmax);
                    if (!(qd >= 0.0)) qd = 0.0;
                    if (qd > (double)qmax) qd = (double)qmax;
                    Q[t] = (uint32_t)qd;
                    T += Q[t];
                }
                if (T > 0 && T <= 0xFFFFFFFFull) {
                    orc_resample(Q, np, orc_resample_offset(cfg->seed, f, k, m, (uint32_t)T), anc);
                } else {
                    for (uint32_t t = 0; t < np; ++t) anc[t] = t;
                    #pragma omp atomic write
                    status = -4;
                }
                if (ta) memcpy(ta, anc, sizeof(uint32_t) * np);
                free(Q);
            } else {
                memcpy(anc, ta, sizeof(uint32_t) * np);
            }
            /* step 8 */
            for (uint32_t t = 0; t < np; ++t) s[base + t] = prop[base + anc[t]];
            free(anc);
            free(w);
        }

        /* steps 9-10: J += log W_k - log N_p and its derivative */
        for (uint32_t f = 0; f < F; ++f) {
            const double *Lf = Lnew + (size_t)f * M;
            double Lg = logsumexp(Lf, M);
            J[f] += Lg - log((double)np);
            if (dJ)
                for (uint32_t m = 0; m < M; ++m) {
                    double pm = (Lg == -INFINITY) ? 0.0 : exp(Lf[m] - Lg);
                    for (int j = 0; j < NTH; ++j)
                        dJ[f * NTH + j] += pm * dLnew[((size_t)f * M + m) * NTH + j];
                }
        }
        memcpy(L, Lnew, sizeof(double) * F * M);
        memcpy(dL, dLnew, sizeof(double) * F * M * NTH);
    }

    orc_destroy(o);
    free(s); free(src); free(prop); free(lam); free(dlam); free(ell); free(dell);
    free(L); free(dL); free(Lnew); free(dLnew); free(pred); free(pi); free(coff); free(P);
    free(origin_pe);
    return status;
}

/* J and dJ/dtheta at the configuration's theta; the choices may be recorded
 * ([K][F], [K][N], [K][N][2]; each pointer nullable). */
int orc_grad(const orc_config *cfg, const double *truth, const float *frames, uint32_t K,
             double *J, double *dJ, uint32_t *tape_nex, uint32_t *tape_anc, int32_t *tape_centre)
{
    return run_frozen(cfg, truth, 0.0, frames, K, 1, tape_nex, tape_anc, tape_centre, J, dJ);
}

/* J with the choices of a tape, at cfg's psf_sigma and q, and every starting
 * intensity shifted by dI0. */
int orc_replay(const orc_config *cfg, const double *truth, double dI0, const float *frames,
               uint32_t K, const uint32_t *tape_nex, const uint32_t *tape_anc,
               const int32_t *tape_centre, double *J)
{
    if (!tape_nex || !tape_anc || !tape_centre) return -1;
    return run_frozen(cfg, truth, dI0, frames, K, 0, (uint32_t *)tape_nex, (uint32_t *)tape_anc,
                      (int32_t *)tape_centre, J, NULL);
}
