/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the cloning
 * (population-dynamics) algorithm for the periodic symmetric simple
 * exclusion process, written from the paper "Efficient characterisation of
 * large deviations using population dynamics" (Brewer, Clark, Bradford, Jack,
 * arXiv:1711.05095).  It exists to check the GPU library against; nothing in
 * the product path may link or call it.  It shares no code, header, table or
 * constant generator with the GPU path.
 *
 * Everything is FP64 and sequential: occupancies are one byte per site, the
 * random streams come from this file's own Philox4x32-10, every loop runs in
 * the order the paper states.
 *
 * What each function follows:
 *   orc_philox      Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel
 *                   random numbers: as easy as 1, 2, 3"), used here in place
 *                   of the paper's per-clone Mersenne Twister (Sec. 6.1).
 *   orc_init        uniform initial configuration at fixed N (the steady
 *                   state of the SSEP, Sec. 3.1), by selection sampling.
 *   orc_step        dynamical stage: continuous-time (BKL) SSEP for one
 *                   interval Delta t (Sec. 4, first paragraph), with
 *                     mode 0: all rates scaled by e^{-s}, cloning factor
 *                             exp(-(1-e^{-s}) * integral of r dt)
 *                             (Sec. 3.2, eq. def-ups-ssep; Sec. 4),
 *                     mode 1: unmodified rates, cloning factor e^{-s K}
 *                             (Sec. 3.1, the biased path weight),
 *                     mode 2: guided rates e^{-s+g} with g from a table
 *                             over bond neighbourhoods, compensating factor
 *                             from eqs. modpdef/upsdef (Sec. 2.2).
 *   orc_select      cloning stage: [eq] (eq. alpha-Ups, Sec. 4.1) or [iid].
 *   orc_resample    cloning stage applied to a population, with the SCGF
 *                   increment ln((1/Nc) sum_i Upsilon_i) (eq. psihat).
 *   orc_run         the whole algorithm: M = t_obs/Delta t repetitions of
 *                   dynamics then cloning (Sec. 2.3), estimators psi-hat
 *                   (eq. psihat) and k-hat (eq. khat, with the 1/Nc the
 *                   printed formula omits; the accumulated K is carried with
 *                   the clone as Sec. 4.2 describes), and both with the
 *                   intervals of a transient left out (Sec. 5.1).
 *   orc_run_lineage the whole algorithm with the origin of every clone
 *                   carried from a chosen interval on: the ancestral lines
 *                   whose end points and starting points have the laws
 *                   p_end and p_ave of Sec. 2.4 (eq. Opave).
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   - bond i joins site i and site (i+1) mod L; it is an allowed hop iff the
 *     two occupancies differ, and each such bond is one hop at rate 1, so the
 *     escape rate r(C) is the number of such bonds (Sec. 3.1);
 *   - the [eq] points are alpha_j = (j + d) Upsilon_T / Nc for j = 0..Nc-1
 *     (the paper's (j+d-1) with 1-based j), and new clone j is pulled from
 *     the old clone whose interval of the cumulative line contains alpha_j;
 *     intervals are half-open [C_{k-1}, C_k).  The comparison is made in
 *     units of the spacing Upsilon_T/Nc: y_k = (C_k * Nc) / Upsilon_T and
 *     "alpha_j lies at or beyond the end of interval k" is y_k <= j + d;
 *   - an event that would straddle the end of the interval is discarded and
 *     redrawn in the next interval with fresh random numbers (memoryless);
 *   - ln mean Upsilon is formed as lmax + log(T / Nc) with
 *     lmax = max_i ln Upsilon_i and T = sum_i exp(ln Upsilon_i - lmax).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                       */
/* ------------------------------------------------------------------ */

/* One Philox4x32 block: ten rounds of the multiply/xor S-box with the
 * published multipliers and Weyl key schedule (SC'11, Sec. 4). */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags: the fourth counter word is tag | (instance << 8). */
enum { ORC_TAG_INIT = 1, ORC_TAG_DYN = 2, ORC_TAG_RESAMPLE = 3, ORC_TAG_IID = 4 };

enum { ORC_MODIFIED = 0, ORC_DIRECT = 1, ORC_GUIDED = 2 };
enum { ORC_SEL_EQ = 0, ORC_SEL_IID = 1 };

typedef struct {
    int32_t L, N;
    double s;
    int64_t Nc;
    double dt;
    int64_t M;            /* number of intervals, t_obs = M * dt */
    uint64_t seed;        /* Philox key */
    uint32_t instance;    /* counter tag, < 2^24 */
    int32_t mode;         /* ORC_MODIFIED / ORC_DIRECT / ORC_GUIDED */
    int32_t selection;    /* ORC_SEL_EQ / ORC_SEL_IID */
    int32_t pad_;
    int64_t burn_in;      /* intervals left out of psi_burn */
    const uint32_t* guide; /* ORC_GUIDED: eg over all 2^13 bond neighbourhoods */
} orc_params;

typedef struct {
    double psi;           /* (1/t_obs) sum_beta ln mean Upsilon^beta */
    double psi_burn;      /* the same sum over beta > burn_in, / ((M - burn_in) dt) */
    double k_hat;         /* sum_j K_j / (Nc L t_obs) of the final population */
    uint64_t hops;        /* every hop performed by every clone */
    int64_t cycles;
    double k_hat_burn;    /* sum_j K'_j / (Nc L (M - burn_in) dt): K' = the hops of the
                             intervals beyond burn_in, carried like K */
} orc_result;

static void draw(const orc_params* p, uint32_t tag, uint32_t c0, uint32_t c1, uint32_t c2,
                 uint32_t x[4])
{
    uint32_t ctr[4] = { c0, c1, c2, tag | (p->instance << 8) };
    uint32_t key[2] = { (uint32_t)p->seed, (uint32_t)(p->seed >> 32) };
    orc_philox(ctr, key, x);
}

/* floor(a * b / 2^64) */
static uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

/* ------------------------------------------------------------------ */
/* Initial condition                                                   */
/* ------------------------------------------------------------------ */

/* Uniform N-subset of the L sites for every clone (selection sampling:
 * site i is taken with probability (N - taken)/(L - i)).  Site i uses the
 * 64-bit number formed from words 2i and 2i+1 of the INIT stream of slot j;
 * the test "u * (L-i) / 2^64 < N - taken" is exact integer arithmetic. */
static void init_clone(const orc_params* p, int64_t slot, uint8_t* n)
{
    const int L = p->L;
    int taken = 0;
    uint32_t x[4];
    for (int i = 0; i < L; ++i) {
        if ((i & 1) == 0)
            draw(p, ORC_TAG_INIT, (uint32_t)(i / 2), (uint32_t)slot, 0u, x);
        uint64_t u = ((i & 1) == 0) ? (((uint64_t)x[0] << 32) | x[1])
                                    : (((uint64_t)x[2] << 32) | x[3]);
        if (mulhi64(u, (uint64_t)(L - i)) < (uint64_t)(p->N - taken)) {
            n[i] = 1;
            ++taken;
        } else {
            n[i] = 0;
        }
    }
}

int orc_init(const orc_params* p, uint8_t* occ, uint64_t* K)
{
    for (int64_t j = 0; j < p->Nc; ++j) {
        init_clone(p, j, occ + (size_t)j * p->L);
        K[j] = 0;
    }
    return 0;
}

/* Initial configuration of a sample of slots. */
int orc_init_slots(const orc_params* p, int64_t n, const int64_t* slots, uint8_t* occ)
{
    for (int64_t i = 0; i < n; ++i) init_clone(p, slots[i], occ + (size_t)i * p->L);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dynamical stage                                                     */
/* ------------------------------------------------------------------ */

static int is_active(const uint8_t* n, int L, int i)
{
    return n[i] != n[(i + 1) % L];
}

/* r(C): the number of bonds whose two sites differ. */
static int escape_count(const uint8_t* n, int L)
{
    int r = 0;
    for (int i = 0; i < L; ++i) r += is_active(n, L, i);
    return r;
}

/* Index of the q-th (0-based, ascending i) active bond. */
static int qth_active_bond(const uint8_t* n, int L, int q)
{
    int seen = 0;
    for (int i = 0; i < L; ++i) {
        if (is_active(n, L, i)) {
            if (seen == q) return i;
            ++seen;
        }
    }
    return -1;
}

/* 13-site window centred on site c, site c-6 in bit 0 ... site c+6 in bit 12. */
static int window13(const uint8_t* n, int L, int c)
{
    int w = 0;
    for (int o = -6; o <= 6; ++o) {
        int site = ((c + o) % L + L) % L;
        w |= (int)n[site] << (o + 6);
    }
    return w;
}

/* ---- guided dynamics (eqs. modpdef, upsdef of Sec. 2.2) ----
 * The guide is a table eg[u] over the 13-site neighbourhood u of a bond
 * (sites b-6 .. b+6, site b-6 in bit 0, so the bond's own sites are bits 6
 * and 7).  The hop across an allowed bond b has rate e^{-s} eg[u_b] 2^-16,
 * i.e. log-ratio g_b = ln(eg[u_b] 2^-16) on top of the modified rate.  With
 * S(C) = sum of eg[u_b] over allowed bonds the escape rate is e^{-s} S 2^-16,
 * and the compensating factor of the interval is
 *     ln Ups = -sum_jumps g - int (r(C) - e^{-s} S(C) 2^-16) dt,
 * which makes the weighted guided trajectories unbiased for ANY table.
 * The jumps are drawn by thinning: proposals come at rate e^{-s} eg_max 2^-16
 * per allowed bond (eg_max the largest entry, so a bound of every controlled
 * rate), each across a uniform allowed bond b, and a proposal is taken with
 * probability eg[u_b] / eg_max, otherwise the configuration stays.  The taken
 * proposals are exactly the jumps of the guided dynamics.  Random numbers of
 * a clone in interval beta: proposal k (counted over the interval from 0)
 * takes Philox block (k, slot, beta, GUIDE): the waiting time from words 0, 1
 * as in the plain dynamics, and the 64-bit bond word bw from words 2, 3; the
 * bond is the q-th allowed one with q = floor(bw r / 2^64), and the rest of
 * that product, a = (bw r) mod 2^64, decides: taken iff
 * floor(a eg_max / 2^64) < eg[u_b].  Given q, a runs over a lattice of
 * spacing r in [0, 2^64), so the acceptance probability is eg/eg_max to
 * within 2 r / 2^64. */
enum { ORC_TAG_GUIDE = 5 };

static uint64_t word_of(uint32_t hi, uint32_t lo) { return ((uint64_t)hi << 32) | lo; }

static uint64_t guided_total(const orc_params* p, const uint8_t* n)
{
    uint64_t S = 0;
    for (int b = 0; b < p->L; ++b)
        if (is_active(n, p->L, b)) S += p->guide[window13(n, p->L, b)];
    return S;
}

static uint32_t guide_max(const orc_params* p)
{
    uint32_t m = 0;
    for (int u = 0; u < 8192; ++u)
        if (p->guide[u] > m) m = p->guide[u];
    return m;
}

static uint32_t step_clone_guided(const orc_params* p, double es, uint32_t egmax, uint32_t beta,
                                  int64_t j, uint8_t* n, double* A_out, double* ell_out)
{
    const int L = p->L;
    const double dt = p->dt;
    const double unit = es * ((double)egmax * 0x1p-16);   /* proposal rate per allowed bond */
    double tau = 0.0, A = 0.0, AS = 0.0, G = 0.0;
    uint32_t kb = 0, k = 0;
    int r = escape_count(n, L);
    uint64_t S = guided_total(p, n);
    while (r > 0) {
        uint32_t x[4];
        draw(p, ORC_TAG_GUIDE, k, (uint32_t)j, beta, x);
        ++k;
        double u = (double)((word_of(x[0], x[1]) >> 11) + 1) * 0x1p-53;
        double E = -log(u);
        double w = E / (unit * (double)r);
        if (tau + w >= dt) {
            A = fma((double)r, dt - tau, A);
            AS = fma((double)S, dt - tau, AS);
            break;
        }
        A = fma((double)r, w, A);
        AS = fma((double)S, w, AS);
        tau = tau + w;
        unsigned __int128 pr = (unsigned __int128)word_of(x[2], x[3]) * (unsigned __int128)r;
        int bond = qth_active_bond(n, L, (int)(uint64_t)(pr >> 64));
        uint32_t e = p->guide[window13(n, L, bond)];
        if (mulhi64((uint64_t)pr, (uint64_t)egmax) >= (uint64_t)e) continue;   /* not taken */
        G += log((double)e * 0x1p-16);
        uint8_t t = n[bond];
        n[bond] = n[(bond + 1) % L];
        n[(bond + 1) % L] = t;
        ++kb;
        r = escape_count(n, L);
        S = guided_total(p, n);
    }
    *A_out = A;
    *ell_out = -G - (A - (es * 0x1p-16) * AS);
    return kb;
}

/* Advance clone j (occupancy n) through interval beta.  Returns the hops. */
static uint32_t step_clone(const orc_params* p, double es, double c, uint32_t beta, int64_t j,
                           uint8_t* n, double* A_out, double* ell_out)
{
    const int L = p->L;
    const double dt = p->dt;
    double tau = 0.0, A = 0.0;
    uint32_t kb = 0, k = 0;
    int r = escape_count(n, L);

    while (r > 0) {
        uint32_t x[4];
        draw(p, ORC_TAG_DYN, k, (uint32_t)j, beta, x);
        ++k;
        /* u in (0, 1] from 53 bits of words 0 and 1 */
        double u = (double)((((uint64_t)x[0] << 21) | (x[1] >> 11)) + 1) * 0x1p-53;
        double E = -log(u);
        double R = (p->mode == ORC_MODIFIED) ? es * (double)r : (double)r;
        double w = E / R;
        if (tau + w >= dt) {
            A = fma((double)r, dt - tau, A);
            break;
        }
        A = fma((double)r, w, A);
        tau = tau + w;
        /* uniform choice among the r allowed hops */
        uint32_t q = (uint32_t)mulhi64(((uint64_t)x[2] << 32) | x[3], (uint64_t)r);
        int bond = qth_active_bond(n, L, (int)q);
        uint8_t t = n[bond];
        n[bond] = n[(bond + 1) % L];
        n[(bond + 1) % L] = t;
        ++kb;
        r = escape_count(n, L);
    }
    *A_out = A;
    *ell_out = (p->mode == ORC_MODIFIED) ? -c * A : -p->s * (double)kb;
    return kb;
}

static uint32_t step_any(const orc_params* p, double es, double c, uint32_t egmax, uint32_t beta,
                         int64_t j, uint8_t* n, double* A_out, double* ell_out)
{
    if (p->mode == ORC_GUIDED) return step_clone_guided(p, es, egmax, beta, j, n, A_out, ell_out);
    return step_clone(p, es, c, beta, j, n, A_out, ell_out);
}

/* One dynamical stage (interval beta >= 1) for the whole population.
 * occ: Nc*L bytes, updated in place.  K: accumulated hops, incremented.
 * Kb, A, ell: per-clone hops, integral of r dt, and ln Upsilon^beta. */
int orc_step(const orc_params* p, uint32_t beta, uint8_t* occ, uint64_t* K, uint32_t* Kb,
             double* A, double* ell)
{
    const double es = exp(-p->s);
    const double c = -expm1(-p->s);
    const uint32_t egmax = (p->mode == ORC_GUIDED) ? guide_max(p) : 0;
    for (int64_t j = 0; j < p->Nc; ++j) {
        uint32_t kb = step_any(p, es, c, egmax, beta, j, occ + (size_t)j * p->L, &A[j], &ell[j]);
        Kb[j] = kb;
        K[j] += kb;
    }
    return 0;
}

/* The dynamical stage for a sample of clones: clone i of the arrays is the
 * clone in slot slots[i] of the population (the slot enters its random
 * stream).  Lets a test check single clones of a population too large to
 * step here in full. */
int orc_step_slots(const orc_params* p, uint32_t beta, int64_t n, const int64_t* slots,
                   uint8_t* occ, uint64_t* K, uint32_t* Kb, double* A, double* ell)
{
    const double es = exp(-p->s);
    const double c = -expm1(-p->s);
    const uint32_t egmax = (p->mode == ORC_GUIDED) ? guide_max(p) : 0;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t kb = step_any(p, es, c, egmax, beta, slots[i], occ + (size_t)i * p->L, &A[i],
                               &ell[i]);
        Kb[i] = kb;
        K[i] += kb;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cloning stage                                                       */
/* ------------------------------------------------------------------ */

/* The [eq] offset d in (0,1) for interval beta: 52 bits of the RESAMPLE
 * stream, centred in its bin. */
double orc_eq_offset(const orc_params* p, uint32_t beta)
{
    uint32_t y[4];
    draw(p, ORC_TAG_RESAMPLE, 0u, 0u, beta, y);
    return ((double)((((uint64_t)y[0]) << 20) | (y[1] >> 12)) + 0.5) * 0x1p-52;
}

/* The [iid] point of new slot j, in units of the spacing: Nc * v, v in (0,1). */
static double iid_point(const orc_params* p, uint32_t beta, int64_t j)
{
    uint32_t y[4];
    draw(p, ORC_TAG_IID, 0u, (uint32_t)j, beta, y);
    double v = ((double)((((uint64_t)y[0]) << 21) | (y[1] >> 11)) + 0.5) * 0x1p-53;
    return v * (double)p->Nc;
}

/* The [iid] points of interval beta for every new slot. */
int orc_iid_points(const orc_params* p, uint32_t beta, double* pts)
{
    for (int64_t j = 0; j < p->Nc; ++j) pts[j] = iid_point(p, beta, j);
    return 0;
}

/* Selection from log-weights ell[0..Nc-1].
 *   selection ORC_SEL_EQ: points j + d (d given), ORC_SEL_IID: points pts[j].
 * Writes anc[j] (the old clone new clone j is pulled from) and returns
 * ln((1/Nc) sum_i exp(ell_i)).  The cumulative key is summed sequentially. */
double orc_select(int64_t Nc, const double* ell, int32_t selection, double d, const double* pts,
                  int32_t* anc)
{
    if (Nc < 1) return 0.0;
    double lmax = ell[0];
    for (int64_t i = 1; i < Nc; ++i)
        if (ell[i] > lmax) lmax = ell[i];
    double* Ck = (double*)malloc(sizeof(double) * (size_t)Nc);
    double acc = 0.0;
    for (int64_t i = 0; i < Nc; ++i) {
        acc += exp(ell[i] - lmax);
        Ck[i] = acc;
    }
    const double T = Ck[Nc - 1];
    /* interval ends in units of the spacing T / Nc */
    for (int64_t i = 0; i < Nc; ++i) Ck[i] = (Ck[i] * (double)Nc) / T;

    for (int64_t j = 0; j < Nc; ++j) {
        /* count of k with y_k <= point (binary search; y is non-decreasing) */
        int64_t lo = 0, hi = Nc; /* answer in [lo, hi] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            int at_or_below;
            if (selection == ORC_SEL_EQ)
                at_or_below = (Ck[mid] - (double)j) <= d; /* exact: see header */
            else
                at_or_below = Ck[mid] <= pts[j];
            if (at_or_below) lo = mid + 1; else hi = mid;
        }
        anc[j] = (int32_t)(lo < Nc ? lo : Nc - 1);
    }
    free(Ck);
    return lmax + log(T / (double)Nc);
}

/* Cloning stage for interval beta: select from ell, then every new clone
 * pulls occupancy and accumulated K from its ancestor. */
double orc_resample(const orc_params* p, uint32_t beta, const uint8_t* occ_old,
                    const uint64_t* K_old, const double* ell, uint8_t* occ_new, uint64_t* K_new,
                    int32_t* anc)
{
    double lmean;
    if (p->selection == ORC_SEL_EQ) {
        lmean = orc_select(p->Nc, ell, ORC_SEL_EQ, orc_eq_offset(p, beta), NULL, anc);
    } else {
        double* pts = (double*)malloc(sizeof(double) * (size_t)p->Nc);
        for (int64_t j = 0; j < p->Nc; ++j) pts[j] = iid_point(p, beta, j);
        lmean = orc_select(p->Nc, ell, ORC_SEL_IID, 0.0, pts, anc);
        free(pts);
    }
    for (int64_t j = 0; j < p->Nc; ++j) {
        memcpy(occ_new + (size_t)j * p->L, occ_old + (size_t)anc[j] * p->L, (size_t)p->L);
        K_new[j] = K_old[anc[j]];
    }
    return lmean;
}

/* ------------------------------------------------------------------ */
/* Whole algorithm                                                     */
/* ------------------------------------------------------------------ */

/* Runs init and M cycles of (dynamics, cloning).  Optional per-interval
 * outputs (may be NULL): lbeta[beta-1] = ln mean Upsilon^beta and
 * mean_kb[beta-1] = population mean of K^beta before cloning.
 *
 * Transient-excluded estimates (the transient of Sec. 5.1): psi_burn sums
 * ln mean Upsilon^beta over beta > burn_in only; for k_hat_burn every clone
 * carries a second count K' that, like K, it inherits from its ancestor at
 * each cloning stage, but that grows only by the hops of intervals
 * beta > burn_in.  Both are divided by the time after burn_in. */
int orc_run(const orc_params* p, orc_result* res, double* lbeta, double* mean_kb)
{
    const int64_t Nc = p->Nc;
    const int L = p->L;
    uint8_t* occ = (uint8_t*)malloc((size_t)Nc * L);
    uint8_t* occ2 = (uint8_t*)malloc((size_t)Nc * L);
    uint64_t* K = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)Nc);
    uint64_t* K2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)Nc);
    uint32_t* Kb = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)Nc);
    double* A = (double*)malloc(sizeof(double) * (size_t)Nc);
    double* ell = (double*)malloc(sizeof(double) * (size_t)Nc);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)Nc);
    uint64_t* Kp = (uint64_t*)calloc((size_t)Nc, sizeof(uint64_t));
    uint64_t* Kp2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)Nc);
    if (!occ || !occ2 || !K || !K2 || !Kb || !A || !ell || !anc || !Kp || !Kp2) return -2;

    orc_init(p, occ, K);
    double psi_sum = 0.0, psi_burn_sum = 0.0;
    uint64_t hops = 0;
    for (int64_t beta = 1; beta <= p->M; ++beta) {
        orc_step(p, (uint32_t)beta, occ, K, Kb, A, ell);
        uint64_t hb = 0;
        for (int64_t j = 0; j < Nc; ++j) hb += Kb[j];
        hops += hb;
        if (beta > p->burn_in)
            for (int64_t j = 0; j < Nc; ++j) Kp[j] += Kb[j];
        double lm = orc_resample(p, (uint32_t)beta, occ, K, ell, occ2, K2, anc);
        for (int64_t j = 0; j < Nc; ++j) Kp2[j] = Kp[anc[j]];
        psi_sum += lm;
        if (beta > p->burn_in) psi_burn_sum += lm;
        if (lbeta) lbeta[beta - 1] = lm;
        if (mean_kb) mean_kb[beta - 1] = (double)hb / (double)Nc;
        uint8_t* to = occ; occ = occ2; occ2 = to;
        uint64_t* tk = K; K = K2; K2 = tk;
        tk = Kp; Kp = Kp2; Kp2 = tk;
    }
    double t_obs = (double)p->M * p->dt;
    double ksum = 0.0, kpsum = 0.0;
    for (int64_t j = 0; j < Nc; ++j) {
        ksum += (double)K[j];
        kpsum += (double)Kp[j];
    }
    const double t_after = (double)(p->M - p->burn_in) * p->dt;
    res->psi = psi_sum / t_obs;
    res->psi_burn = (p->M > p->burn_in) ? psi_burn_sum / t_after : 0.0;
    res->k_hat = ksum / ((double)Nc * (double)L * t_obs);
    res->k_hat_burn = (p->M > p->burn_in) ? kpsum / ((double)Nc * (double)L * t_after) : 0.0;
    res->hops = hops;
    res->cycles = p->M;
    free(occ); free(occ2); free(K); free(K2); free(Kb); free(A); free(ell); free(anc);
    free(Kp); free(Kp2);
    return 0;
}

/* Ancestral lines (Sec. 2.4): runs init and M cycles like orc_run.  After the
 * cloning stage of interval beta0 (1 <= beta0 <= M) the population is copied
 * to occ_b0 and every clone is marked as its own origin; from then on a clone
 * inherits its ancestor's origin at every cloning stage.  At the end occ_end
 * holds the final population (after the last cloning stage) and origin[j]
 * the slot, at beta0, of the ancestor of final clone j.  occ_b0 and occ_end:
 * Nc * L bytes; origin: Nc entries. */
int orc_run_lineage(const orc_params* p, int64_t beta0, uint8_t* occ_b0, uint8_t* occ_end,
                    int32_t* origin)
{
    const int64_t Nc = p->Nc;
    const int L = p->L;
    if (beta0 < 1 || beta0 > p->M) return -1;
    uint8_t* occ = (uint8_t*)malloc((size_t)Nc * L);
    uint8_t* occ2 = (uint8_t*)malloc((size_t)Nc * L);
    uint64_t* K = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)Nc);
    uint64_t* K2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)Nc);
    uint32_t* Kb = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)Nc);
    double* A = (double*)malloc(sizeof(double) * (size_t)Nc);
    double* ell = (double*)malloc(sizeof(double) * (size_t)Nc);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)Nc);
    int32_t* org2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)Nc);
    if (!occ || !occ2 || !K || !K2 || !Kb || !A || !ell || !anc || !org2) return -2;

    orc_init(p, occ, K);
    for (int64_t beta = 1; beta <= p->M; ++beta) {
        orc_step(p, (uint32_t)beta, occ, K, Kb, A, ell);
        orc_resample(p, (uint32_t)beta, occ, K, ell, occ2, K2, anc);
        if (beta > beta0) {
            for (int64_t j = 0; j < Nc; ++j) org2[j] = origin[anc[j]];
            memcpy(origin, org2, sizeof(int32_t) * (size_t)Nc);
        }
        uint8_t* to = occ; occ = occ2; occ2 = to;
        uint64_t* tk = K; K = K2; K2 = tk;
        if (beta == beta0) {
            memcpy(occ_b0, occ, (size_t)Nc * L);
            for (int64_t j = 0; j < Nc; ++j) origin[j] = (int32_t)j;
        }
    }
    memcpy(occ_end, occ, (size_t)Nc * L);
    free(occ); free(occ2); free(K); free(K2); free(Kb); free(A); free(ell); free(anc);
    free(org2);
    return 0;
}
