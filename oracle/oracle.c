/*
 * oracle.c -- plain, slow, float64 CPU oracle for the MC-MD / MDAS force and
 * energy path (Cherniavskyi, Fathizadeh, Elber, Tieleman, arXiv 2005.08348).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no source with the GPU library.
 *
 * Everything is float64, scalar, written to be checked by eye against the
 * paper and the textbook definitions it relies on:
 *   - potential: potential-shifted Lennard-Jones 12-6 with a 1.1 nm cutoff
 *     and reaction-field electrostatics (Section 3, Methods); harmonic bonds
 *     and cosine-squared angles of the Martini model (Section 3);
 *   - MC-MD exchange move with the Metropolis test (Section 2, Eq. 1);
 *   - MDAS alchemical trajectory with linear coupling U(l)=(1-l)U_A + l U_B,
 *     its work (Section 2, Eq. 2) and acceptance (Section 2, Eq. 3);
 *   - Langevin dynamics in the BAOAB splitting (the paper's engine is not
 *     specified beyond "MD"; this is the reading used throughout);
 *   - Philox4x32-10 counter-based random numbers (Salmon, Moraes, Dror,
 *     Shaw, SC'11), written from that paper's definition.
 *
 * Functions whose result has no independent pin are marked "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O_KB 0.00831446261815324      /* kJ/mol/K */
#define O_FELEC 138.935458            /* kJ mol^-1 nm e^-2, 1/(4 pi eps0) */
#define O_MAXEXCL 8
#define O_PI 3.14159265358979323846

/* random stream ids (fourth counter word) */
enum { ST_LANGEVIN = 0, ST_SWAP_DRAW = 1, ST_SWAP_ACCEPT = 2,
       ST_MDAS_SELECT = 3, ST_MDAS_ACCEPT = 4, ST_VRESCALE = 5, ST_BARO = 6 };

typedef struct {
    /* kinds */
    int nk;
    int *kn, *koff, *ktype, *kfam;
    double *kq, *km;
    int *knb, *kboff, *bi, *bj;
    double *bb0, *bk;
    int *kna, *kaoff, *ai, *aj, *ak;
    double *acos0, *akk;
    /* molecules */
    int nm;
    int *mkind, *mfirst;
    /* beads */
    int n;
    int *bmol, *bloc;
    int *nexcl, *excl;      /* per bead up to O_MAXEXCL bonded partners */
    /* force field */
    int nt;
    double *c6, *c12;
    double box[3], rc, eps_r, eps_rf, krf, crf, fpre;
    /* dynamics */
    double dt, kT, gamma;
    uint64_t seed;
    /* state */
    double *x, *v, *f;
    int64_t step, batch, cycle;
    long n_fe;
    /* scratch */
    int *mk_tmp;
    double *f_tmp;
    double *f_slab;          /* per-slab force buffers of the nonbonded loop */
    /* ensemble: 0 Langevin BAOAB, 1 velocity Verlet + stochastic velocity
     * rescaling of two coupling groups */
    int ensemble;
    double tau_t;
    int kgroup[64];          /* coupling group of each kind */
    /* exchange regions (leaflets): 0 partners anywhere, 1 within the
     * region of X, 2 in the other region */
    int xmode;
    int* region;             /* [nm] 0 or 1 */
    /* semi-isotropic pressure coupling every baro_nst steps (0: off):
     * baro_kind 0 stochastic cell rescaling, 1 Parrinello-Rahman */
    int baro_nst, baro_kind;
    /* ktopo[k1 * nk + k2]: kinds k1 and k2 differ in their bonded terms */
    int* ktopo;
    double p_ref, kappa, tau_p;   /* kJ mol^-1 nm^-3, its inverse, ps */
    double box_v[3];              /* Parrinello-Rahman box velocity, nm/ps */
    double w_box;                 /* Parrinello-Rahman box mass, amu */
    /* MDAS lambda path: 0 linear in the end-state energies (Eq. 2),
     * 1 soft-core LJ of the changed beads (Eq. 4, shift sc_delta nm^2) */
    int mdas_path;
    double sc_delta;
} osys;

/* ------------------------------------------------------------ Philox4x32-10 */
/* One round: two 32x32->64 multiplies of counter words 0 and 2 by the
 * published multipliers, the high halves xor-ed with the other two counter
 * words and the key; the key is bumped by the Weyl constants between rounds. */
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (r < 9) { k0 += W0; k1 += W1; }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void o_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    philox4x32_10(ctr, key, out);
}

static void draw(const osys* s, uint32_t index, int64_t c, uint32_t stream,
                 uint32_t w[4])
{
    uint32_t ctr[4] = { index, (uint32_t)((uint64_t)c & 0xffffffffu),
                        (uint32_t)((uint64_t)c >> 32), stream };
    uint32_t key[2] = { (uint32_t)(s->seed & 0xffffffffu), (uint32_t)(s->seed >> 32) };
    philox4x32_10(ctr, key, w);
}

/* uniform on [0,1) with 53 random bits */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* index in [0, n) */
static uint32_t pick(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* three standard normals from one Philox block (Box-Muller) */
static void gauss3(const uint32_t w[4], double g[3])
{
    const double two32 = 4294967296.0, twopi = 6.283185307179586476925286766559;
    double u1 = ((double)w[0] + 1.0) / two32, u2 = (double)w[1] / two32;
    double u3 = ((double)w[2] + 1.0) / two32, u4 = (double)w[3] / two32;
    double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    g[0] = r1 * cos(twopi * u2);
    g[1] = r1 * sin(twopi * u2);
    g[2] = r2 * cos(twopi * u4);
}

void o_gauss3(const uint32_t* w, double* g) { gauss3(w, g); }

/* ------------------------------------------------------------------- create */
static void* xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

static void set_bead_tables(osys* s)
{
    for (int m = 0; m < s->nm; ++m) {
        int k = s->mkind[m];
        for (int b = 0; b < s->kn[k]; ++b) {
            s->bmol[s->mfirst[m] + b] = m;
            s->bloc[s->mfirst[m] + b] = b;
        }
    }
}

osys* o_create(int nk, const int* kn, const int* ktype, const double* kq,
               const double* km, const int* kfam,
               const int* knb, const int* bond_ij, const double* bb0, const double* bk,
               const int* kna, const int* ang_ijk, const double* ath0_deg, const double* akk,
               int nm, const int* mkind,
               int nt, const double* eps, const double* sig,
               const double* box, double rc, double eps_r, double eps_rf,
               double dt, double T, double gamma, uint64_t seed,
               const double* x, const double* v)
{
    osys* s = (osys*)xcalloc(1, sizeof(osys));
    s->nk = nk;
    s->kn = (int*)xcalloc(nk, sizeof(int));
    s->koff = (int*)xcalloc(nk, sizeof(int));
    s->kfam = (int*)xcalloc(nk, sizeof(int));
    s->knb = (int*)xcalloc(nk, sizeof(int));
    s->kboff = (int*)xcalloc(nk, sizeof(int));
    s->kna = (int*)xcalloc(nk, sizeof(int));
    s->kaoff = (int*)xcalloc(nk, sizeof(int));
    int tb = 0, tbo = 0, tan = 0;
    for (int k = 0; k < nk; ++k) {
        s->kn[k] = kn[k]; s->koff[k] = tb; tb += kn[k];
        s->kfam[k] = kfam[k];
        s->knb[k] = knb[k]; s->kboff[k] = tbo; tbo += knb[k];
        s->kna[k] = kna[k]; s->kaoff[k] = tan; tan += kna[k];
    }
    s->ktype = (int*)xcalloc(tb, sizeof(int));
    s->kq = (double*)xcalloc(tb, sizeof(double));
    s->km = (double*)xcalloc(tb, sizeof(double));
    memcpy(s->ktype, ktype, sizeof(int) * tb);
    memcpy(s->kq, kq, sizeof(double) * tb);
    memcpy(s->km, km, sizeof(double) * tb);
    s->bi = (int*)xcalloc(tbo, sizeof(int));
    s->bj = (int*)xcalloc(tbo, sizeof(int));
    s->bb0 = (double*)xcalloc(tbo, sizeof(double));
    s->bk = (double*)xcalloc(tbo, sizeof(double));
    for (int b = 0; b < tbo; ++b) {
        s->bi[b] = bond_ij[2 * b]; s->bj[b] = bond_ij[2 * b + 1];
        s->bb0[b] = bb0[b]; s->bk[b] = bk[b];
    }
    s->ai = (int*)xcalloc(tan, sizeof(int));
    s->aj = (int*)xcalloc(tan, sizeof(int));
    s->ak = (int*)xcalloc(tan, sizeof(int));
    s->acos0 = (double*)xcalloc(tan, sizeof(double));
    s->akk = (double*)xcalloc(tan, sizeof(double));
    for (int a = 0; a < tan; ++a) {
        s->ai[a] = ang_ijk[3 * a]; s->aj[a] = ang_ijk[3 * a + 1]; s->ak[a] = ang_ijk[3 * a + 2];
        s->acos0[a] = cos(ath0_deg[a] * (3.14159265358979323846 / 180.0));
        s->akk[a] = akk[a];
    }
    s->ktopo = (int*)xcalloc((size_t)nk * nk, sizeof(int));
    for (int k1 = 0; k1 < nk; ++k1)
        for (int k2 = 0; k2 < nk; ++k2) {
            int dif = s->knb[k1] != s->knb[k2] || s->kna[k1] != s->kna[k2];
            for (int b = 0; !dif && b < s->knb[k1]; ++b) {
                int p = s->kboff[k1] + b, q = s->kboff[k2] + b;
                dif = s->bi[p] != s->bi[q] || s->bj[p] != s->bj[q] || s->bb0[p] != s->bb0[q] ||
                      s->bk[p] != s->bk[q];
            }
            for (int a = 0; !dif && a < s->kna[k1]; ++a) {
                int p = s->kaoff[k1] + a, q = s->kaoff[k2] + a;
                dif = s->ai[p] != s->ai[q] || s->aj[p] != s->aj[q] || s->ak[p] != s->ak[q] ||
                      s->acos0[p] != s->acos0[q] || s->akk[p] != s->akk[q];
            }
            s->ktopo[k1 * nk + k2] = dif;
        }
    s->nm = nm;
    s->mkind = (int*)xcalloc(nm, sizeof(int));
    s->region = (int*)xcalloc(nm, sizeof(int));
    s->mfirst = (int*)xcalloc(nm, sizeof(int));
    s->mk_tmp = (int*)xcalloc(nm, sizeof(int));
    int n = 0;
    for (int m = 0; m < nm; ++m) {
        s->mkind[m] = mkind[m]; s->mfirst[m] = n; n += kn[mkind[m]];
    }
    s->n = n;
    s->bmol = (int*)xcalloc(n, sizeof(int));
    s->bloc = (int*)xcalloc(n, sizeof(int));
    set_bead_tables(s);
    /* exclusions: beads joined by a bond of their molecule (nrexcl = 1).
     * A molecule of a swap family whose kinds differ in their bonds (a
     * topology-changing exchange) excludes the pairs bonded in any kind of
     * the family, so that its nonbonded pair set does not depend on its
     * current kind. */
    s->nexcl = (int*)xcalloc(n, sizeof(int));
    s->excl = (int*)xcalloc((size_t)n * O_MAXEXCL, sizeof(int));
    for (int m = 0; m < nm; ++m) {
        int k0 = s->mkind[m], f0 = s->mfirst[m];
        for (int k = 0; k < nk; ++k) {
            if (k != k0 && (s->kfam[k0] < 0 || s->kfam[k] != s->kfam[k0])) continue;
            for (int b = 0; b < s->knb[k]; ++b) {
                int i = f0 + s->bi[s->kboff[k] + b], j = f0 + s->bj[s->kboff[k] + b];
                int dup = 0;
                for (int e = 0; e < s->nexcl[i]; ++e)
                    if (s->excl[(size_t)i * O_MAXEXCL + e] == j) dup = 1;
                if (dup) continue;
                if (s->nexcl[i] < O_MAXEXCL) s->excl[(size_t)i * O_MAXEXCL + s->nexcl[i]++] = j;
                if (s->nexcl[j] < O_MAXEXCL) s->excl[(size_t)j * O_MAXEXCL + s->nexcl[j]++] = i;
            }
        }
    }
    s->nt = nt;
    s->c6 = (double*)xcalloc((size_t)nt * nt, sizeof(double));
    s->c12 = (double*)xcalloc((size_t)nt * nt, sizeof(double));
    for (int a = 0; a < nt * nt; ++a) {
        double s6 = pow(sig[a], 6.0);
        s->c6[a] = 4.0 * eps[a] * s6;
        s->c12[a] = 4.0 * eps[a] * s6 * s6;
    }
    for (int d = 0; d < 3; ++d) s->box[d] = box[d];
    s->rc = rc; s->eps_r = eps_r; s->eps_rf = eps_rf;
    /* reaction field with dielectric eps_rf beyond the cutoff */
    if (isinf(eps_rf)) s->krf = 1.0 / (2.0 * rc * rc * rc);
    else s->krf = (eps_rf - eps_r) / ((2.0 * eps_rf + eps_r) * rc * rc * rc);
    s->crf = 1.0 / rc + s->krf * rc * rc;
    s->fpre = O_FELEC / eps_r;
    s->dt = dt; s->kT = O_KB * T; s->gamma = gamma; s->seed = seed;
    s->x = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->v = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->f = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->f_tmp = (double*)xcalloc((size_t)3 * n, sizeof(double));
    memcpy(s->x, x, sizeof(double) * 3 * n);
    if (v) memcpy(s->v, v, sizeof(double) * 3 * n);
    return s;
}

void o_destroy(osys* s)
{
    if (!s) return;
    void* p[] = { s->kn, s->koff, s->ktype, s->kfam, s->kq, s->km, s->knb, s->kboff,
                  s->bi, s->bj, s->bb0, s->bk, s->kna, s->kaoff, s->ai, s->aj, s->ak,
                  s->acos0, s->akk, s->mkind, s->mfirst, s->bmol, s->bloc, s->nexcl,
                  s->excl, s->c6, s->c12, s->x, s->v, s->f, s->mk_tmp, s->f_tmp, s->region, s->f_slab,
                  s->ktopo };
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
    free(s);
}

int o_n(const osys* s) { return s->n; }
void o_get_state(const osys* s, double* x, double* v, double* f, int* mkind, int64_t* ctr)
{
    if (x) memcpy(x, s->x, sizeof(double) * 3 * s->n);
    if (v) memcpy(v, s->v, sizeof(double) * 3 * s->n);
    if (f) memcpy(f, s->f, sizeof(double) * 3 * s->n);
    if (mkind) memcpy(mkind, s->mkind, sizeof(int) * s->nm);
    if (ctr) { ctr[0] = s->step; ctr[1] = s->batch; ctr[2] = s->cycle; ctr[3] = s->n_fe; }
}
void o_set_state(osys* s, const double* x, const double* v, const int* mkind,
                 const int64_t* ctr)
{
    if (x) memcpy(s->x, x, sizeof(double) * 3 * s->n);
    if (v) memcpy(s->v, v, sizeof(double) * 3 * s->n);
    if (mkind) memcpy(s->mkind, mkind, sizeof(int) * s->nm);
    if (ctr) { s->step = ctr[0]; s->batch = ctr[1]; s->cycle = ctr[2]; }
}

/* --------------------------------------------------------------- geometry */
/* minimum-image separation x_i - x_j, rounding the image index to nearest
 * (ties to even). */
static void min_image(const osys* s, const double* xi, const double* xj, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double t = xi[a] - xj[a];
        t -= s->box[a] * nearbyint(t / s->box[a]);
        d[a] = t;
    }
}

static double dist2(const double d[3])
{
    double r2 = d[0] * d[0];
    r2 = r2 + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    return r2;
}

static int excluded(const osys* s, int i, int j)
{
    for (int e = 0; e < s->nexcl[i]; ++e)
        if (s->excl[(size_t)i * O_MAXEXCL + e] == j) return 1;
    return 0;
}

static inline int btype_k(const osys* s, const int* mk, int b)
{
    return s->ktype[s->koff[mk[s->bmol[b]]] + s->bloc[b]];
}
static inline double bq_k(const osys* s, const int* mk, int b)
{
    return s->kq[s->koff[mk[s->bmol[b]]] + s->bloc[b]];
}
static inline double bmass(const osys* s, int b)
{
    return s->km[s->koff[s->mkind[s->bmol[b]]] + s->bloc[b]];
}

/* Pair energy and scalar force -dV/dr / r for types ti,tj and charges qi,qj
 * at squared distance r2 < rc^2.
 *   V_LJ = C12/r^12 - C6/r^6 - (C12/rc^12 - C6/rc^6)
 *   V_RF = f qi qj (1/r + k_rf r^2 - c_rf)                                  */
static void pair_term(const osys* s, int ti, int tj, double qi, double qj,
                      double r2, double* vlj, double* vrf, double* fscal)
{
    double c6 = s->c6[ti * s->nt + tj], c12 = s->c12[ti * s->nt + tj];
    double r = sqrt(r2);
    double ir2 = 1.0 / r2, ir6 = ir2 * ir2 * ir2;
    double rc6 = pow(s->rc, 6.0), rc12 = rc6 * rc6;
    double qq = s->fpre * qi * qj;
    *vlj = c12 * ir6 * ir6 - c6 * ir6 - (c12 / rc12 - c6 / rc6);
    *vrf = qq * (1.0 / r + s->krf * r2 - s->crf);
    *fscal = (12.0 * c12 * ir6 * ir6 - 6.0 * c6 * ir6) * ir2
           + qq * (1.0 / (r2 * r) - 2.0 * s->krf);
}

void o_pair_term(const osys* s, int ti, int tj, double qi, double qj, double r2, double* out)
{
    pair_term(s, ti, tj, qi, qj, r2, &out[0], &out[1], &out[2]);
}

/* --------------------------------------------------------------- cell grid */
typedef struct { int nc[3]; int* head; int* next; } cgrid;

static void grid_build(const osys* s, double edge_min, cgrid* g)
{
    int ntot = 1;
    for (int a = 0; a < 3; ++a) {
        int c = (int)floor(s->box[a] / edge_min);
        if (c < 3) c = 3;   /* fewer than 3 cells: every cell is a neighbour */
        g->nc[a] = c; ntot *= c;
    }
    g->head = (int*)malloc(sizeof(int) * ntot);
    g->next = (int*)malloc(sizeof(int) * (s->n ? s->n : 1));
    for (int c = 0; c < ntot; ++c) g->head[c] = -1;
    for (int i = s->n - 1; i >= 0; --i) {
        int ci[3];
        for (int a = 0; a < 3; ++a) {
            double u = s->x[3 * i + a] / s->box[a];
            u -= floor(u);
            int c = (int)floor(u * g->nc[a]);
            if (c >= g->nc[a]) c = g->nc[a] - 1;
            if (c < 0) c = 0;
            ci[a] = c;
        }
        int c = (ci[0] * g->nc[1] + ci[1]) * g->nc[2] + ci[2];
        g->next[i] = g->head[c];
        g->head[c] = i;
    }
}

static void grid_free(cgrid* g) { free(g->head); free(g->next); }

/* Visit every unordered non-excluded pair i<j with d^2 < cut2.  With only 3
 * cells along an axis the offsets -1 and +1 are distinct cells, so no pair is
 * visited twice; the box must be at least three cutoffs wide for the cell
 * path, otherwise the all-pairs path is used. */
typedef void (*pair_fn)(osys* s, int i, int j, const double d[3], double r2, void* ctx);

static int cells_usable(const osys* s, double cut, int use_cells)
{
    int ok = use_cells;
    for (int a = 0; a < 3; ++a) if (s->box[a] < 3.0 * cut) ok = 0;
    return ok;
}

/* The pairs whose first bead lies in the cells cx in [cx0, cx1) of grid g. */
static void for_pairs_slab(osys* s, const cgrid* g, double cut2, int cx0, int cx1, pair_fn fn,
                           void* ctx)
{
    for (int cx = cx0; cx < cx1; ++cx)
    for (int cy = 0; cy < g->nc[1]; ++cy)
    for (int cz = 0; cz < g->nc[2]; ++cz) {
        int c = (cx * g->nc[1] + cy) * g->nc[2] + cz;
        for (int i = g->head[c]; i >= 0; i = g->next[i]) {
            for (int ox = -1; ox <= 1; ++ox)
            for (int oy = -1; oy <= 1; ++oy)
            for (int oz = -1; oz <= 1; ++oz) {
                int nx = (cx + ox + g->nc[0]) % g->nc[0];
                int ny = (cy + oy + g->nc[1]) % g->nc[1];
                int nz = (cz + oz + g->nc[2]) % g->nc[2];
                int cn = (nx * g->nc[1] + ny) * g->nc[2] + nz;
                for (int j = g->head[cn]; j >= 0; j = g->next[j]) {
                    if (j <= i) continue;
                    double d[3];
                    min_image(s, &s->x[3 * i], &s->x[3 * j], d);
                    double r2 = dist2(d);
                    if (r2 < cut2 && !excluded(s, i, j)) fn(s, i, j, d, r2, ctx);
                }
            }
        }
    }
}

static void for_pairs(osys* s, double cut, int use_cells, pair_fn fn, void* ctx)
{
    double cut2 = cut * cut;
    if (!cells_usable(s, cut, use_cells)) {
        for (int i = 0; i < s->n; ++i)
            for (int j = i + 1; j < s->n; ++j) {
                double d[3];
                min_image(s, &s->x[3 * i], &s->x[3 * j], d);
                double r2 = dist2(d);
                if (r2 < cut2 && !excluded(s, i, j)) fn(s, i, j, d, r2, ctx);
            }
        return;
    }
    cgrid g;
    grid_build(s, cut, &g);
    for_pairs_slab(s, &g, cut2, 0, g.nc[0], fn, ctx);
    grid_free(&g);
}

/* ------------------------------------------------------------ nonbonded */
typedef struct { const int* mk; double* f; double elj, erf; long npairs; } nb_ctx;

static void nb_pair(osys* s, int i, int j, const double d[3], double r2, void* vctx)
{
    nb_ctx* c = (nb_ctx*)vctx;
    double vlj, vrf, fs;
    pair_term(s, btype_k(s, c->mk, i), btype_k(s, c->mk, j),
              bq_k(s, c->mk, i), bq_k(s, c->mk, j), r2, &vlj, &vrf, &fs);
    c->elj += vlj; c->erf += vrf; c->npairs++;
    if (c->f)
        for (int a = 0; a < 3; ++a) {
            c->f[3 * i + a] += fs * d[a];
            c->f[3 * j + a] -= fs * d[a];
        }
}

/* ---------------------------------------------------------------- bonded */
static void bonded(const osys* s, const int* mk, double* f, double* eb, double* ea)
{
    double Eb = 0.0, Ea = 0.0;
    for (int m = 0; m < s->nm; ++m) {
        int k = mk[m], f0 = s->mfirst[m];
        for (int b = 0; b < s->knb[k]; ++b) {
            int bb = s->kboff[k] + b;
            int i = f0 + s->bi[bb], j = f0 + s->bj[bb];
            double d[3];
            min_image(s, &s->x[3 * i], &s->x[3 * j], d);
            double r = sqrt(dist2(d));
            double dr = r - s->bb0[bb];
            Eb += 0.5 * s->bk[bb] * dr * dr;
            if (f) {
                double fs = -s->bk[bb] * dr / r;   /* force on i along d */
                for (int a = 0; a < 3; ++a) { f[3 * i + a] += fs * d[a]; f[3 * j + a] -= fs * d[a]; }
            }
        }
        for (int t = 0; t < s->kna[k]; ++t) {
            int aa = s->kaoff[k] + t;
            int i = f0 + s->ai[aa], j = f0 + s->aj[aa], l = f0 + s->ak[aa];
            double u[3], w[3];
            min_image(s, &s->x[3 * i], &s->x[3 * j], u);   /* x_i - x_j */
            min_image(s, &s->x[3 * l], &s->x[3 * j], w);   /* x_k - x_j */
            double uu = dist2(u), ww = dist2(w);
            double nu = sqrt(uu), nw = sqrt(ww);
            double uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
            double cth = uw / (nu * nw);
            double dc = cth - s->acos0[aa];
            Ea += 0.5 * s->akk[aa] * dc * dc;
            if (f) {
                double pre = -s->akk[aa] * dc;
                for (int a = 0; a < 3; ++a) {
                    double dci = w[a] / (nu * nw) - cth * u[a] / uu;   /* d cos / d x_i */
                    double dck = u[a] / (nu * nw) - cth * w[a] / ww;   /* d cos / d x_k */
                    f[3 * i + a] += pre * dci;
                    f[3 * l + a] += pre * dck;
                    f[3 * j + a] -= pre * (dci + dck);
                }
            }
        }
    }
    *eb = Eb; *ea = Ea;
}

/* Energies and forces for molecule kinds mk.  e = {lj, rf, bond, angle}.
 * use_cells selects the cell-list pair loop (identical pair set). */
/* The cell path visits the pairs in O_NSLAB slabs of cells along x, each
 * with its own energy sums and force buffer, and adds the slabs in slab
 * order: the result is the same whether the slabs run one after another or
 * on several threads (OpenMP, when the oracle is built with it). */
#define O_NSLAB 16
static long energy_forces(osys* s, const int* mk, double* f, double e[4], int use_cells)
{
    if (f) memset(f, 0, sizeof(double) * 3 * s->n);
    double eb, ea;
    if (!cells_usable(s, s->rc, use_cells)) {
        nb_ctx c = { mk, f, 0.0, 0.0, 0 };
        for_pairs(s, s->rc, 0, nb_pair, &c);
        bonded(s, mk, f, &eb, &ea);
        e[0] = c.elj; e[1] = c.erf; e[2] = eb; e[3] = ea;
        return c.npairs;
    }
    cgrid g;
    grid_build(s, s->rc, &g);
    const size_t n3 = 3 * (size_t)s->n;
    if (f && !s->f_slab) s->f_slab = (double*)malloc(sizeof(double) * n3 * O_NSLAB);
    nb_ctx c[O_NSLAB];
    const double rc2 = s->rc * s->rc;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) if (s->n >= 20000)
#endif
    for (int k = 0; k < O_NSLAB; ++k) {
        double* fk = f ? s->f_slab + n3 * k : NULL;
        if (fk) memset(fk, 0, sizeof(double) * n3);
        c[k].mk = mk; c[k].f = fk; c[k].elj = 0.0; c[k].erf = 0.0; c[k].npairs = 0;
        for_pairs_slab(s, &g, rc2, k * g.nc[0] / O_NSLAB, (k + 1) * g.nc[0] / O_NSLAB, nb_pair,
                       &c[k]);
    }
    grid_free(&g);
    long np = 0;
    double elj = 0.0, erf = 0.0;
    for (int k = 0; k < O_NSLAB; ++k) {
        elj += c[k].elj; erf += c[k].erf; np += c[k].npairs;
        if (f)
            for (size_t q = 0; q < n3; ++q) f[q] += s->f_slab[n3 * k + q];
    }
    bonded(s, mk, f, &eb, &ea);
    e[0] = elj; e[1] = erf; e[2] = eb; e[3] = ea;
    return np;
}

/* Number of threads the slabs of the nonbonded loop and the sampled forces
 * may use (1 without OpenMP); n <= 0 leaves the current setting.  Returns
 * the setting in force. */
int o_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* public: energies/forces of the current state.  out_e = {lj, rf, bond,
 * angle, kinetic}; returns the number of non-excluded pairs inside r_c. */
long o_energy_forces(osys* s, double* f, double* out_e, int use_cells)
{
    double e[4];
    long np = energy_forces(s, s->mkind, f, e, use_cells);
    double ke = 0.0;
    for (int i = 0; i < s->n; ++i) {
        double m = bmass(s, i);
        ke += 0.5 * m * (s->v[3 * i] * s->v[3 * i] + s->v[3 * i + 1] * s->v[3 * i + 1]
                         + s->v[3 * i + 2] * s->v[3 * i + 2]);
    }
    if (out_e) { for (int a = 0; a < 4; ++a) out_e[a] = e[a]; out_e[4] = ke; }
    return np;
}

/* ------------------------------------------------------ virial, pressure */
/* Pressure tensor diagonal (needed by the paper's barostat, Methods):
 * P_aa V = sum_i m_i v_ia^2 + W_aa, with the virial W_aa the sum over
 * interactions of (separation)_a (force)_a: for a pair or bond, the
 * minimum-image separation r_i - r_j times the force on i; for an angle
 * i-j-k, (r_i - r_j) F_i + (r_k - r_j) F_k (the three forces sum to zero).
 * W_aa equals -dU/d eps for the affine stretch x_a -> (1 + eps) x_a of all
 * beads and of the box. */
typedef struct { const int* mk; double w[3], wabs[3]; } vir_ctx;

static void vir_pair(osys* s, int i, int j, const double d[3], double r2, void* vctx)
{
    vir_ctx* c = (vir_ctx*)vctx;
    double vlj, vrf, fs;
    pair_term(s, btype_k(s, c->mk, i), btype_k(s, c->mk, j),
              bq_k(s, c->mk, i), bq_k(s, c->mk, j), r2, &vlj, &vrf, &fs);
    for (int a = 0; a < 3; ++a) {
        c->w[a] += d[a] * fs * d[a];
        c->wabs[a] += fabs(d[a] * fs * d[a]);
    }
}

/* w[0..2] = W_aa, w[3..5] = sum m v_a^2, w[6..8] = sum of |term| of W_aa
 * (the scale of rounding errors in a reduced-precision evaluation) */
void o_virial(osys* s, double* w, int use_cells)
{
    vir_ctx c = { s->mkind, { 0.0, 0.0, 0.0 }, { 0.0, 0.0, 0.0 } };
    for_pairs(s, s->rc, use_cells, vir_pair, &c);
    for (int m = 0; m < s->nm; ++m) {
        int k = s->mkind[m], f0 = s->mfirst[m];
        for (int b = 0; b < s->knb[k]; ++b) {
            int bb = s->kboff[k] + b;
            int i = f0 + s->bi[bb], j = f0 + s->bj[bb];
            double d[3];
            min_image(s, &s->x[3 * i], &s->x[3 * j], d);
            double r = sqrt(dist2(d));
            double fs = -s->bk[bb] * (r - s->bb0[bb]) / r;
            for (int a = 0; a < 3; ++a) {
                c.w[a] += d[a] * fs * d[a];
                c.wabs[a] += fabs(d[a] * fs * d[a]);
            }
        }
        for (int t = 0; t < s->kna[k]; ++t) {
            int aa = s->kaoff[k] + t;
            int i = f0 + s->ai[aa], j = f0 + s->aj[aa], l = f0 + s->ak[aa];
            double u[3], v[3];
            min_image(s, &s->x[3 * i], &s->x[3 * j], u);
            min_image(s, &s->x[3 * l], &s->x[3 * j], v);
            double uu = dist2(u), vv = dist2(v), nu = sqrt(uu), nv = sqrt(vv);
            double cth = (u[0] * v[0] + u[1] * v[1] + u[2] * v[2]) / (nu * nv);
            double pre = -s->akk[aa] * (cth - s->acos0[aa]);
            for (int a = 0; a < 3; ++a) {
                double fi = pre * (v[a] / (nu * nv) - cth * u[a] / uu);
                double fk = pre * (u[a] / (nu * nv) - cth * v[a] / vv);
                c.w[a] += u[a] * fi + v[a] * fk;
                c.wabs[a] += fabs(u[a] * fi) + fabs(v[a] * fk);
            }
        }
    }
    for (int a = 0; a < 3; ++a) { w[a] = c.w[a]; w[3 + a] = 0.0; w[6 + a] = c.wabs[a]; }
    for (int i = 0; i < s->n; ++i) {
        double m = bmass(s, i);
        for (int a = 0; a < 3; ++a) w[3 + a] += m * s->v[3 * i + a] * s->v[3 * i + a];
    }
}

/* Force on selected beads by direct summation over every other bead
 * (O(N) per bead; for sampled checks on large systems).  Also returns, per
 * bead, the smallest |r^2 - rc^2| over its pairs so that callers can set
 * aside beads whose pair set depends on rounding at the cutoff. */
void o_forces_on(osys* s, int nsel, const int* sel, double* fout, double* near_cut)
{
    double rc2 = s->rc * s->rc;
    int maxkn = 1;
    for (int k = 0; k < s->nk; ++k) if (s->kn[k] > maxkn) maxkn = s->kn[k];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) if ((double)nsel * s->n >= 1e7)
#endif
    for (int q = 0; q < nsel; ++q) {
        int i = sel[q];
        double fx = 0, fy = 0, fz = 0, nc = 1e300;
        for (int j = 0; j < s->n; ++j) {
            if (j == i || excluded(s, i, j)) continue;
            double d[3];
            min_image(s, &s->x[3 * i], &s->x[3 * j], d);
            double r2 = dist2(d);
            double gap = fabs(r2 - rc2);
            if (gap < nc) nc = gap;
            if (r2 >= rc2) continue;
            double vlj, vrf, fs;
            pair_term(s, btype_k(s, s->mkind, i), btype_k(s, s->mkind, j),
                      bq_k(s, s->mkind, i), bq_k(s, s->mkind, j), r2, &vlj, &vrf, &fs);
            fx += fs * d[0]; fy += fs * d[1]; fz += fs * d[2];
        }
        /* bonded terms touching bead i: evaluate its molecule's terms */
        int m = s->bmol[i], k = s->mkind[m], f0 = s->mfirst[m];
        double* fm = (double*)malloc(sizeof(double) * 3 * maxkn);
        int nb = s->kn[k];
        memset(fm, 0, sizeof(double) * 3 * nb);
        for (int b = 0; b < s->knb[k]; ++b) {
            int bb = s->kboff[k] + b;
            int li = s->bi[bb], lj = s->bj[bb];
            double d[3];
            min_image(s, &s->x[3 * (f0 + li)], &s->x[3 * (f0 + lj)], d);
            double r = sqrt(dist2(d)), dr = r - s->bb0[bb];
            double fs = -s->bk[bb] * dr / r;
            for (int a = 0; a < 3; ++a) { fm[3 * li + a] += fs * d[a]; fm[3 * lj + a] -= fs * d[a]; }
        }
        for (int t = 0; t < s->kna[k]; ++t) {
            int aa = s->kaoff[k] + t;
            int li = s->ai[aa], lj = s->aj[aa], lk = s->ak[aa];
            double u[3], w[3];
            min_image(s, &s->x[3 * (f0 + li)], &s->x[3 * (f0 + lj)], u);
            min_image(s, &s->x[3 * (f0 + lk)], &s->x[3 * (f0 + lj)], w);
            double uu = dist2(u), ww = dist2(w), nu = sqrt(uu), nw = sqrt(ww);
            double cth = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / (nu * nw);
            double pre = -s->akk[aa] * (cth - s->acos0[aa]);
            for (int a = 0; a < 3; ++a) {
                double dci = w[a] / (nu * nw) - cth * u[a] / uu;
                double dck = u[a] / (nu * nw) - cth * w[a] / ww;
                fm[3 * li + a] += pre * dci;
                fm[3 * lk + a] += pre * dck;
                fm[3 * lj + a] -= pre * (dci + dck);
            }
        }
        int lb = s->bloc[i];
        fout[3 * q] = fx + fm[3 * lb];
        fout[3 * q + 1] = fy + fm[3 * lb + 1];
        fout[3 * q + 2] = fz + fm[3 * lb + 2];
        if (near_cut) near_cut[q] = nc;
        free(fm);
    }
}

/* ---------------------------------------------------------------- pair set */
typedef struct { int* out; long cap, n; } ps_ctx;
static void ps_pair(osys* s, int i, int j, const double d[3], double r2, void* vctx)
{
    (void)s; (void)d; (void)r2;
    ps_ctx* c = (ps_ctx*)vctx;
    if (c->n < c->cap) { c->out[2 * c->n] = i; c->out[2 * c->n + 1] = j; }
    c->n++;
}

/* all non-excluded pairs i<j with float64 d^2 < rlist^2 (unordered) */
long o_pairset(osys* s, double rlist, int* out, long cap, int use_cells)
{
    ps_ctx c = { out, cap, 0 };
    for_pairs(s, rlist, use_cells, ps_pair, &c);
    return c.n;
}

/* ------------------------------------------------------------- dynamics */
/* ---------------------------------------------------- soft-core lambda path */
/* Eq. 4 with sigma^2 / (r^2 + delta (1 - mu)) as the base (the printed
 * formula's sigma over r^2 read dimensionally), written with c6 = 4 eps
 * sigma^6, c12 = 4 eps sigma^12: V = mu (c12 / s^6 - c6 / s^3), s = r^2 +
 * delta (1 - mu); at mu = 1 the plain 12-6 form, at mu = 0 nothing, finite
 * at r = 0 for mu < 1.  As the paper's Martini runs shift the LJ potential to
 * zero at the cutoff, the soft-core term is shifted by its own value at r_c
 * (the plain shifted form at mu = 1).  fscal = -dV/dr / r. */
static void sc_lj(double c6, double c12, double r2, double mu, double delta, double rc2,
                  double* v, double* fscal)
{
    double sh = delta * (1.0 - mu);
    double s3 = r2 + sh, i3 = 1.0 / (s3 * s3 * s3);
    double c3 = rc2 + sh, ic3 = 1.0 / (c3 * c3 * c3);
    *v = mu * (c12 * i3 * i3 - c6 * i3) - mu * (c12 * ic3 * ic3 - c6 * ic3);
    *fscal = mu * (12.0 * c12 * i3 * i3 - 6.0 * c6 * i3) / s3;
}

void o_sc_lj(double c6, double c12, double r2, double mu, double delta, double rc, double* out)
{
    sc_lj(c6, c12, r2, mu, delta, rc * rc, &out[0], &out[1]);
}

/* The alchemical state at lambda on the soft-core path, for end-state kinds
 * mk_b: a pair with no changed bead (same type and charge in both states)
 * keeps its plain terms; a pair with a changed bead takes the A-state LJ at
 * mu = 1 - lambda and the B-state LJ at mu = lambda, both soft-core, and the
 * reaction field of the charge product (1 - lambda) q_i q_j |A + lambda
 * q_i q_j |B.  Bonded terms are (1 - lambda) U_A + lambda U_B (the same
 * terms in both states unless the exchange changes the topology).
 * U_0 = U_A and U_1 = U_B exactly. */
typedef struct { const int* mk_b; const char* chg; double lam; double* f; double u; } sc_ctx;

static void sc_pair(osys* s, int i, int j, const double d[3], double r2, void* vctx)
{
    sc_ctx* c = (sc_ctx*)vctx;
    double v, fs;
    if (!c->chg[i] && !c->chg[j]) {
        double vlj, vrf;
        pair_term(s, btype_k(s, s->mkind, i), btype_k(s, s->mkind, j),
                  bq_k(s, s->mkind, i), bq_k(s, s->mkind, j), r2, &vlj, &vrf, &fs);
        v = vlj + vrf;
    } else {
        const int ta = btype_k(s, s->mkind, i), tb = btype_k(s, s->mkind, j);
        const int ua = btype_k(s, c->mk_b, i), ub = btype_k(s, c->mk_b, j);
        double va, fa, vb, fb;
        sc_lj(s->c6[ta * s->nt + tb], s->c12[ta * s->nt + tb], r2, 1.0 - c->lam, s->sc_delta,
              s->rc * s->rc, &va, &fa);
        sc_lj(s->c6[ua * s->nt + ub], s->c12[ua * s->nt + ub], r2, c->lam, s->sc_delta,
              s->rc * s->rc, &vb, &fb);
        const double qq = (1.0 - c->lam) * bq_k(s, s->mkind, i) * bq_k(s, s->mkind, j)
                        + c->lam * bq_k(s, c->mk_b, i) * bq_k(s, c->mk_b, j);
        const double r = sqrt(r2), pre = s->fpre * qq;
        v = va + vb + pre * (1.0 / r + s->krf * r2 - s->crf);
        fs = fa + fb + pre * (1.0 / (r2 * r) - 2.0 * s->krf);
    }
    c->u += v;
    if (c->f)
        for (int a = 0; a < 3; ++a) { c->f[3 * i + a] += fs * d[a]; c->f[3 * j + a] -= fs * d[a]; }
}

static double sc_energy_forces(osys* s, const int* mk_b, double lam, double* f)
{
    char* chg = (char*)calloc(s->n, 1);
    for (int i = 0; i < s->n; ++i)
        chg[i] = btype_k(s, s->mkind, i) != btype_k(s, mk_b, i) || bq_k(s, s->mkind, i) != bq_k(s, mk_b, i);
    if (f) memset(f, 0, sizeof(double) * 3 * s->n);
    sc_ctx c = { mk_b, chg, lam, f, 0.0 };
    for_pairs(s, s->rc, 1, sc_pair, &c);
    double eb, ea, ub = 0.0;
    int topo = 0;
    for (int m = 0; m < s->nm; ++m) topo |= s->ktopo[s->mkind[m] * s->nk + mk_b[m]];
    if (!topo || lam == 0.0 || lam == 1.0) {
        bonded(s, lam == 0.0 ? s->mkind : mk_b, f, &eb, &ea);
        ub = eb + ea;
    } else {
        double* fb = f ? (double*)calloc((size_t)3 * s->n, sizeof(double)) : NULL;
        bonded(s, s->mkind, fb, &eb, &ea);
        ub += (1.0 - lam) * (eb + ea);
        if (f) for (int q = 0; q < 3 * s->n; ++q) { f[q] += (1.0 - lam) * fb[q]; fb[q] = 0.0; }
        bonded(s, mk_b, fb, &eb, &ea);
        ub += lam * (eb + ea);
        if (f) for (int q = 0; q < 3 * s->n; ++q) f[q] += lam * fb[q];
        free(fb);
    }
    free(chg);
    return c.u + ub;
}

/* U at lambda on the soft-core path for exchanging the given pairs */
double o_sc_energy(osys* s, int n_pairs, const int* pairs, double lam)
{
    int* mk_b = (int*)malloc(sizeof(int) * s->nm);
    memcpy(mk_b, s->mkind, sizeof(int) * s->nm);
    for (int p = 0; p < n_pairs; ++p) {
        int X = pairs[2 * p], Y = pairs[2 * p + 1];
        mk_b[X] = s->mkind[Y]; mk_b[Y] = s->mkind[X];
    }
    double u = sc_energy_forces(s, mk_b, lam, NULL);
    free(mk_b);
    return u;
}

void o_set_mdas_path(osys* s, int path, double delta) { s->mdas_path = path; s->sc_delta = delta; }

static double force_eval(osys* s, const int* mk_b, double lam, double* f)
{
    /* F(lam) = (1-lam) F_A + lam F_B ; returns U(lam) */
    double e[4];
    if (mk_b && s->mdas_path == 1) {
        s->n_fe++;
        return sc_energy_forces(s, mk_b, lam, f);
    }
    if (!mk_b || lam == 0.0) {
        energy_forces(s, s->mkind, f, e, 1);
        s->n_fe++;
        return e[0] + e[1] + e[2] + e[3];
    }
    double eb[4];
    energy_forces(s, s->mkind, s->f_tmp, e, 1);
    energy_forces(s, mk_b, f, eb, 1);
    s->n_fe++;
    for (int i = 0; i < 3 * s->n; ++i) f[i] = (1.0 - lam) * s->f_tmp[i] + lam * f[i];
    return (1.0 - lam) * (e[0] + e[1] + e[2] + e[3]) + lam * (eb[0] + eb[1] + eb[2] + eb[3]);
}

/* U(lambda) and F(lambda) = -grad U(lambda) of the MDAS path in force (the
 * linear coupling of Eq. 2, or the soft-core path of Eq. 4) for exchanging
 * the given pairs, at the current coordinates: what the dynamics of an
 * alchemical trajectory feel at coupling lambda (not counted as an FE). */
double o_hybrid_energy_forces(osys* s, int n_pairs, const int* pairs, double lam, double* f)
{
    int* mk_b = (int*)malloc(sizeof(int) * s->nm);
    memcpy(mk_b, s->mkind, sizeof(int) * s->nm);
    for (int p = 0; p < n_pairs; ++p) {
        int X = pairs[2 * p], Y = pairs[2 * p + 1];
        mk_b[X] = s->mkind[Y]; mk_b[Y] = s->mkind[X];
    }
    double u = force_eval(s, mk_b, lam, f);
    s->n_fe--;
    free(mk_b);
    return u;
}

/* Refresh the stored forces for the current state (needed after set_state). */
void o_refresh_forces(osys* s) { force_eval(s, NULL, 0.0, s->f); s->n_fe--; }

/* One BAOAB step at coupling lam (mk_b = end-state kinds or NULL):
 *   v += dt/2 F/m; x += dt/2 v; v = c1 v + c2 sqrt(kT/m) xi; x += dt/2 v;
 *   F = F(x); v += dt/2 F/m.
 * The stored forces on entry are those of the current x at the current lam. */
static void baoab(osys* s, const int* mk_b, double lam)
{
    double h = 0.5 * s->dt;
    double c1 = exp(-s->gamma * s->dt), c2 = sqrt(1.0 - c1 * c1);
    for (int i = 0; i < s->n; ++i) {
        double m = bmass(s, i), sg = sqrt(s->kT / m);
        uint32_t w[4];
        double g[3];
        draw(s, (uint32_t)i, s->step, ST_LANGEVIN, w);
        gauss3(w, g);
        for (int a = 0; a < 3; ++a) {
            double v = s->v[3 * i + a] + h * s->f[3 * i + a] / m;
            double x = s->x[3 * i + a] + h * v;
            v = c1 * v + c2 * sg * g[a];
            x = x + h * v;
            s->v[3 * i + a] = v;
            s->x[3 * i + a] = x;
        }
    }
    force_eval(s, mk_b, lam, s->f);
    for (int i = 0; i < s->n; ++i) {
        double m = bmass(s, i);
        for (int a = 0; a < 3; ++a) s->v[3 * i + a] += h * s->f[3 * i + a] / m;
    }
    s->step++;
}

/* ------------------------------------------------- velocity rescaling (f2) */
/* The paper's runs keep the temperature with stochastic velocity rescaling
 * (Methods).  After each velocity Verlet step the kinetic energy K of each
 * coupling group is moved to K' by one step of the stochastic dynamics of
 * Bussi, Donadio and Parrinello (J. Chem. Phys. 126, 014101, 2007), with
 * c = exp(-dt / tau_t), target Kt = Nf kT / 2 and Nf = 3 (beads in the
 * group):  K' = K + (1 - c) (Kt (R1^2 + S) / Nf - K)
 *              + 2 R1 sqrt(c (1 - c) K Kt / Nf),
 * R1 standard normal, S chi-squared with Nf - 1 degrees of freedom; the
 * velocities of the group are multiplied by alpha = +-sqrt(K' / K), negative
 * when R1 + sqrt(c Nf K / ((1 - c) Kt)) < 0.  Random numbers: Philox
 * stream 5 with counter = the step index; block (group << 16) gives R1 from
 * its first two words, blocks (group << 16) + 1 + t the t-th attempt of the
 * gamma sampler below. */

/* one standard normal from two words (Box-Muller, cosine branch) */
static double normal1(uint32_t a, uint32_t b)
{
    const double two32 = 4294967296.0, twopi = 6.283185307179586476925286766559;
    double u1 = ((double)a + 1.0) / two32, u2 = (double)b / two32;
    return sqrt(-2.0 * log(u1)) * cos(twopi * u2);
}

/* Gamma(a, 1), a >= 1, by Marsaglia and Tsang (ACM TOMS 26, 363, 2000):
 * d = a - 1/3, c = 1/sqrt(9 d); draw x standard normal and u uniform until
 * v = (1 + c x)^3 > 0 and log u < x^2 / 2 + d - d v + d log v; return d v.
 * At most 64 attempts (then d, which has probability ~0 to matter). */
static double gamma_mt(const osys* s, int g, double a, int64_t ctr)
{
    const double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
    for (int t = 0; t < 64; ++t) {
        uint32_t w[4];
        draw(s, (uint32_t)((g << 16) + 1 + t), ctr, ST_VRESCALE, w);
        const double x = normal1(w[0], w[1]);
        const double u = u53(w[2], w[3]);
        const double y = 1.0 + c * x;
        if (y <= 0.0) continue;
        const double v = y * y * y;
        if (log(u) < 0.5 * x * x + d - d * v + d * log(v)) return d * v;
    }
    return d;
}

static double vr_alpha(const osys* s, int g, double K, double nf, int64_t ctr)
{
    if (!(K > 0.0) || !(nf >= 3.0)) return 1.0;
    const double c = exp(-s->dt / s->tau_t);
    const double kt = 0.5 * nf * s->kT;
    uint32_t w[4];
    draw(s, (uint32_t)(g << 16), ctr, ST_VRESCALE, w);
    const double r1 = normal1(w[0], w[1]);
    const double sch = 2.0 * gamma_mt(s, g, 0.5 * (nf - 1.0), ctr);
    const double kn = K + (1.0 - c) * (kt * (r1 * r1 + sch) / nf - K) +
                      2.0 * r1 * sqrt(c * (1.0 - c) * K * kt / nf);
    double al = sqrt(kn / K);
    if (r1 + sqrt(c * nf * K / ((1.0 - c) * kt)) < 0.0) al = -al;
    return al;
}

/* one velocity Verlet step (BAOAB without the O part) and the rescaling of
 * each group with the counter of that step */
static void vv_vrescale(osys* s, const int* mk_b, double lam)
{
    const double g0 = s->gamma;
    s->gamma = 0.0;
    const int64_t ctr = s->step;    /* the thermostat draws with this step's counter */
    baoab(s, mk_b, lam);            /* advances s->step */
    s->gamma = g0;
    double K[2] = { 0.0, 0.0 }, nf[2] = { 0.0, 0.0 };
    for (int i = 0; i < s->n; ++i) {
        const int g = s->kgroup[s->mkind[s->bmol[i]]];
        const double m = bmass(s, i);
        const double* v = s->v + 3 * i;
        K[g] += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        nf[g] += 3.0;
    }
    const double al[2] = { vr_alpha(s, 0, K[0], nf[0], ctr), vr_alpha(s, 1, K[1], nf[1], ctr) };
    for (int i = 0; i < s->n; ++i) {
        const double a = al[s->kgroup[s->mkind[s->bmol[i]]]];
        for (int q = 0; q < 3; ++q) s->v[3 * i + q] *= a;
    }
}

void o_set_ensemble(osys* s, int ensemble, double tau_t, const int* kind_group)
{
    s->ensemble = ensemble;
    s->tau_t = tau_t;
    for (int k = 0; k < s->nk && k < 64; ++k) s->kgroup[k] = kind_group ? (kind_group[k] != 0) : 0;
}

void o_set_exchange_regions(osys* s, int mode, const int* region)
{
    s->xmode = mode;
    for (int m = 0; m < s->nm; ++m) s->region[m] = region ? (region[m] != 0) : 0;
}

/* the statistics pins use these directly: n draws at counters ctr0 .. ctr0 + n - 1 */
void o_gamma_mt(osys* s, int g, double a, int64_t ctr0, int n, double* out)
{
    for (int t = 0; t < n; ++t) out[t] = gamma_mt(s, g, a, ctr0 + t);
}
void o_vr_alpha(osys* s, int g, double K, double nf, int64_t ctr0, int n, double* out)
{
    for (int t = 0; t < n; ++t) out[t] = vr_alpha(s, g, K, nf, ctr0 + t);
}

/* one MD step of the selected ensemble (at coupling lam for MDAS segments) */
static void md_one(osys* s, const int* mk_b, double lam)
{
    if (s->ensemble == 1) vv_vrescale(s, mk_b, lam);
    else baoab(s, mk_b, lam);
}

/* ---------------------------------------------------- pressure coupling */
/* The paper keeps 1 bar with a semi-isotropic barostat (Methods): the box
 * lengths in the membrane plane (x and y together) and normal to it (z)
 * respond separately.  Here the box follows stochastic cell rescaling
 * (Bernetti and Bussi, J. Chem. Phys. 153, 114107, 2020) in two log-strains,
 * e_A = ln(Lx Ly) and e_z = ln Lz, each an overdamped Langevin process
 * whose stationary law is p(e_A, e_z) ~ V^(N+1) exp(-(U + P0 V) / kT), the
 * isothermal-isobaric law of positions with box lengths Lx = Ly and Lz
 * drawn uniformly in (Lx Ly, Lz).  With P_A = (N kT + (W_xx + W_yy) / 2) / V
 * and P_z = (N kT + W_zz) / V, one Euler-Maruyama (Ito) step over t = nst dt is
 *   d e = -(kappa / tau_p) (P0 - P) t + sqrt(2 kappa kT t / (V tau_p)) xi
 * per strain: the drift -D (d Psi / d e + 1) that makes exp(-Psi) stationary
 * for the diffusion D = kappa kT / (V tau_p), which falls as 1/V (Psi =
 * (U + P0 V) / kT - (N + 1) ln V; the Jacobian term and the Ito term of the
 * V-dependent noise cancel).  x and y scale by exp(d e_A / 2), z by
 * exp(d e_z), about the
 * origin, with the box; velocities are left to the thermostat.  xi: Box-
 * Muller normals from Philox stream 6, block 0, counter = the step index
 * after the step that triggers the coupling. */
static void couple_pressure(osys* s)
{
    double w[9];
    o_virial(s, w, 1);
    const double V = s->box[0] * s->box[1] * s->box[2];
    const double nkt = (double)s->n * s->kT;
    const double pa = (nkt + 0.5 * (w[0] + w[1])) / V, pz = (nkt + w[2]) / V;
    const double t = s->baro_nst * s->dt;
    uint32_t r[4];
    draw(s, 0u, s->step, ST_BARO, r);
    const double xa = normal1(r[0], r[1]), xz = normal1(r[2], r[3]);
    const double drift = s->kappa / s->tau_p * t, amp = sqrt(2.0 * s->kappa * s->kT * t / (V * s->tau_p));
    const double dea = -drift * (s->p_ref - pa) + amp * xa;
    const double dez = -drift * (s->p_ref - pz) + amp * xz;
    const double mu[3] = { exp(0.5 * dea), exp(0.5 * dea), exp(dez) };
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < 3; ++a) s->x[3 * i + a] *= mu[a];
    for (int a = 0; a < 3; ++a) s->box[a] *= mu[a];
    force_eval(s, NULL, 0.0, s->f);   /* forces of the rescaled configuration */
    s->n_fe--;                        /* a refresh, not a step */
}

/* Parrinello-Rahman pressure coupling, the paper's barostat (Methods;
 * Parrinello and Rahman, J. Appl. Phys. 52, 7182 (1981)), for a box that
 * stays rectangular, semi-isotropic.  Positions are r = L s (s scaled
 * coordinates, L the box lengths) and the integrator's velocities are the
 * peculiar ones, u_a = L_a ds_a/dt.  The extended Hamiltonian
 *   H = sum_i m_i |u_i|^2 / 2 + U + P0 V + (W / 2) sum_a (dL_a/dt)^2
 * gives W d2L_a/dt2 = V (P_aa - P0) / L_a with P_aa V = sum_i m_i u_ia^2 + W_aa
 * (the pressure tensor of o_virial), and du_a/dt = F_a / m - (dL_a/dt / L_a) u_a:
 * a change of L_a at fixed s scales r_a by L'_a / L_a and u_a by L_a / L'_a.
 * Semi-isotropic: x and y are both driven by (P_xx + P_yy) / 2, which for a
 * box with L_x = L_y is the same Hamiltonian with L_x = L_y held equal.  Box
 * mass: W = 3 tau_p^2 L_max / (4 pi^2 beta) with beta the compressibility
 * and L_max the longest edge when the coupling is switched on (the usual
 * choice, under which a system of compressibility beta swings with period
 * tau_p), held fixed so that H is conserved without a thermostat.
 * Discretisation, every nst steps (t = nst dt), after the step that ends the
 * interval: the box velocity takes the impulse of the whole interval at the
 * current pressure, dL_a/dt += t V (P_aa - P0) / (W L_a), then the box moves
 * L'_a = L_a + t dL_a/dt with r and u scaled as above, and the forces of the
 * new configuration are evaluated.  The particles step at fixed box in
 * between.  H is conserved to first order in t (tests pin its convergence). */
static void couple_pr(osys* s)
{
    double w[9];
    o_virial(s, w, 1);
    const double V = s->box[0] * s->box[1] * s->box[2];
    const double t = s->baro_nst * s->dt;
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = (w[3 + a] + w[a]) / V;
    const double pxy = 0.5 * (p[0] + p[1]);
    const double drive[3] = { pxy - s->p_ref, pxy - s->p_ref, p[2] - s->p_ref };
    double mu[3];
    for (int a = 0; a < 3; ++a) {
        s->box_v[a] += t * V * drive[a] / (s->w_box * s->box[a]);
        mu[a] = (s->box[a] + t * s->box_v[a]) / s->box[a];
    }
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < 3; ++a) {
            s->x[3 * i + a] *= mu[a];
            s->v[3 * i + a] /= mu[a];
        }
    for (int a = 0; a < 3; ++a) s->box[a] *= mu[a];
    force_eval(s, NULL, 0.0, s->f);   /* forces of the new configuration */
    s->n_fe--;                        /* a refresh, not a step */
}

void o_set_barostat(osys* s, int nst, double p_ref, double kappa, double tau_p)
{
    s->baro_nst = nst > 0 ? nst : 0;
    s->baro_kind = 0;
    s->p_ref = p_ref; s->kappa = kappa; s->tau_p = tau_p;
}

/* Parrinello-Rahman coupling every nst steps (0: off); p_ref in
 * kJ mol^-1 nm^-3, beta in its inverse, tau_p in ps.  The box velocity
 * starts at zero and W is fixed from the current box. */
void o_set_barostat_pr(osys* s, int nst, double p_ref, double beta, double tau_p)
{
    s->baro_nst = nst > 0 ? nst : 0;
    s->baro_kind = 1;
    s->p_ref = p_ref; s->kappa = beta; s->tau_p = tau_p;
    double lmax = fmax(s->box[0], fmax(s->box[1], s->box[2]));
    s->w_box = 3.0 * tau_p * tau_p * lmax / (4.0 * O_PI * O_PI * beta);
    for (int a = 0; a < 3; ++a) s->box_v[a] = 0.0;
}

/* Box velocity (nm/ps, may be NULL) and the box's terms of the conserved
 * Parrinello-Rahman energy, P0 V + (W / 2) sum_a (dL_a/dt)^2 (kJ/mol). */
double o_barostat_state(const osys* s, double* box_v)
{
    if (box_v) for (int a = 0; a < 3; ++a) box_v[a] = s->box_v[a];
    double k = 0.0;
    for (int a = 0; a < 3; ++a) k += 0.5 * s->w_box * s->box_v[a] * s->box_v[a];
    return s->p_ref * s->box[0] * s->box[1] * s->box[2] + k;
}

void o_set_box_velocity(osys* s, const double* box_v)
{
    for (int a = 0; a < 3; ++a) s->box_v[a] = box_v[a];
}

void o_get_box(const osys* s, double* box) { for (int a = 0; a < 3; ++a) box[a] = s->box[a]; }

void o_md_step(osys* s, int nsteps)
{
    for (int t = 0; t < nsteps; ++t) {
        md_one(s, NULL, 0.0);
        if (s->baro_nst > 0 && s->step % s->baro_nst == 0) {
            if (s->baro_kind == 1) couple_pr(s);
            else couple_pressure(s);
        }
    }
}

/* Capped steepest descent: each bead moves by alpha F_i, shortened to at most
 * `cap` nm.  Used only to relax synthetic start structures.  Pinned by the
 * LJ minimum at 2^(1/6) sigma of an isolated pair, a lone bond relaxing to
 * b0 and the exact cap from an overlap; no GPU result is compared with it. */
void o_minimize(osys* s, int n_iter, double alpha, double cap)
{
    double e[4];
    for (int it = 0; it < n_iter; ++it) {
        energy_forces(s, s->mkind, s->f, e, 1);
        for (int i = 0; i < s->n; ++i) {
            double d[3], l2 = 0.0;
            for (int a = 0; a < 3; ++a) { d[a] = alpha * s->f[3 * i + a]; l2 += d[a] * d[a]; }
            double l = sqrt(l2);
            double sc = (l > cap) ? cap / l : 1.0;
            for (int a = 0; a < 3; ++a) {
                double x = s->x[3 * i + a] + sc * d[a];
                x -= s->box[a] * floor(x / s->box[a]);
                s->x[3 * i + a] = x;
            }
        }
    }
    energy_forces(s, s->mkind, s->f, e, 1);
}

/* ------------------------------------------------------- exchange moves */
/* beads (local indices) whose (type, charge) differ between kinds a and b */
static int changed_locals(const osys* s, int ka, int kb, int* loc)
{
    int n = 0;
    for (int b = 0; b < s->kn[ka]; ++b) {
        int oa = s->koff[ka] + b, ob = s->koff[kb] + b;
        if (s->ktype[oa] != s->ktype[ob] || s->kq[oa] != s->kq[ob]) loc[n++] = b;
    }
    return n;
}

/* May molecule m partner X (kind kx, family fam) under the exchange mode?
 * Mode 0: any molecule of the family of another kind.  Mode 1: the same,
 * within X's region (leaflet): leaflet compositions never change.  Mode 2
 * (the interleaflet move the paper proposes in its Discussion): any
 * molecule of the family in the other region, whatever its kind.  Partner
 * sets of modes 0 and 1 depend on the kinds, but the swap leaves the counts
 * they are drawn from unchanged; the mode-2 set does not depend on the
 * kinds at all, and a partner of X's own kind is a trial that changes
 * nothing.  Either way the chance to propose a pair equals that of the
 * reverse proposal, so the Metropolis test of Eq. 1 needs no correction. */
static int may_partner(const osys* s, int m, int x, int kx, int fam)
{
    if (s->kfam[s->mkind[m]] != fam) return 0;
    if (s->xmode == 2) return s->region[m] != s->region[x];
    if (s->mkind[m] == kx) return 0;
    return s->xmode == 1 ? s->region[m] == s->region[x] : 1;
}

/* Draw one candidate pair (X, Y) from Philox words w: X uniform over the
 * molecules of any swap family, Y uniform (ascending molecule id) over X's
 * partners (may_partner).  Returns 0 if X has none. */
static int draw_pair(const osys* s, const uint32_t w[4], int* X, int* Y)
{
    int nsw = 0;
    for (int m = 0; m < s->nm; ++m) if (s->kfam[s->mkind[m]] >= 0) nsw++;
    if (nsw == 0) return 0;
    uint32_t ix = pick(w[0], (uint32_t)nsw);
    int x = -1, c = 0;
    for (int m = 0; m < s->nm; ++m)
        if (s->kfam[s->mkind[m]] >= 0) { if ((uint32_t)c == ix) { x = m; break; } c++; }
    int fam = s->kfam[s->mkind[x]], kx = s->mkind[x];
    int nother = 0;
    for (int m = 0; m < s->nm; ++m)
        if (may_partner(s, m, x, kx, fam)) nother++;
    if (nother == 0) return 0;
    uint32_t iy = pick(w[1], (uint32_t)nother);
    int y = -1;
    c = 0;
    for (int m = 0; m < s->nm; ++m)
        if (may_partner(s, m, x, kx, fam)) {
            if ((uint32_t)c == iy) { y = m; break; }
            c++;
        }
    *X = x; *Y = y;
    return 1;
}

/* Bonded energy of molecule m if it had kind k, at the current coordinates. */
static double mol_bonded_energy(const osys* s, int m, int k)
{
    double Eb = 0.0, Ea = 0.0;
    int f0 = s->mfirst[m];
    for (int b = 0; b < s->knb[k]; ++b) {
        int bb = s->kboff[k] + b;
        double d[3];
        min_image(s, &s->x[3 * (f0 + s->bi[bb])], &s->x[3 * (f0 + s->bj[bb])], d);
        double dr = sqrt(dist2(d)) - s->bb0[bb];
        Eb += 0.5 * s->bk[bb] * dr * dr;
    }
    for (int t = 0; t < s->kna[k]; ++t) {
        int aa = s->kaoff[k] + t;
        double u[3], w[3];
        min_image(s, &s->x[3 * (f0 + s->ai[aa])], &s->x[3 * (f0 + s->aj[aa])], u);
        min_image(s, &s->x[3 * (f0 + s->ak[aa])], &s->x[3 * (f0 + s->aj[aa])], w);
        double cth = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / (sqrt(dist2(u)) * sqrt(dist2(w)));
        double dc = cth - s->acos0[aa];
        Ea += 0.5 * s->akk[aa] * dc * dc;
    }
    return Eb + Ea;
}

/* U(after) - U(before) for exchanging the kinds of molecules X and Y: the
 * pair terms that involve a changed bead, plus, when the kinds differ in
 * their bonded terms (a topology-changing exchange), the bonded energies of
 * X and Y in their new kinds minus those in their old ones. */
static double delta_u_pair(osys* s, int X, int Y)
{
    int kx = s->mkind[X], ky = s->mkind[Y];
    int loc[64];
    int nl = changed_locals(s, kx, ky, loc);
    int ch[128], nch = 0;
    for (int q = 0; q < nl; ++q) { ch[nch++] = s->mfirst[X] + loc[q]; }
    for (int q = 0; q < nl; ++q) { ch[nch++] = s->mfirst[Y] + loc[q]; }
    int* mk = s->mk_tmp;
    memcpy(mk, s->mkind, sizeof(int) * s->nm);
    mk[X] = ky; mk[Y] = kx;
    double rc2 = s->rc * s->rc, du = 0.0;
    for (int a = 0; a < nch; ++a) {
        int i = ch[a];
        for (int j = 0; j < s->n; ++j) {
            if (j == i || excluded(s, i, j)) continue;
            int jchanged = 0;
            for (int b = 0; b < nch; ++b) if (ch[b] == j) jchanged = 1;
            if (jchanged && j < i) continue;   /* count changed-changed pairs once */
            double d[3];
            min_image(s, &s->x[3 * i], &s->x[3 * j], d);
            double r2 = dist2(d);
            if (r2 >= rc2) continue;
            double v1a, v1b, v0a, v0b, fs;
            pair_term(s, btype_k(s, mk, i), btype_k(s, mk, j), bq_k(s, mk, i), bq_k(s, mk, j),
                      r2, &v1a, &v1b, &fs);
            pair_term(s, btype_k(s, s->mkind, i), btype_k(s, s->mkind, j),
                      bq_k(s, s->mkind, i), bq_k(s, s->mkind, j), r2, &v0a, &v0b, &fs);
            du += (v1a + v1b) - (v0a + v0b);
        }
    }
    if (s->ktopo[kx * s->nk + ky])
        du += (mol_bonded_energy(s, X, ky) + mol_bonded_energy(s, Y, kx))
            - (mol_bonded_energy(s, X, kx) + mol_bonded_energy(s, Y, ky));
    return du;
}

double o_delta_u_pair(osys* s, int X, int Y) { return delta_u_pair(s, X, Y); }

/* U(after) - U(before) from two full recomputations (for checking). */
double o_delta_u_full(osys* s, int X, int Y)
{
    int* mk = (int*)malloc(sizeof(int) * s->nm);
    memcpy(mk, s->mkind, sizeof(int) * s->nm);
    mk[X] = s->mkind[Y]; mk[Y] = s->mkind[X];
    double e0[4], e1[4];
    energy_forces(s, s->mkind, NULL, e0, 0);
    energy_forces(s, mk, NULL, e1, 0);
    free(mk);
    return (e1[0] + e1[1] + e1[2] + e1[3]) - (e0[0] + e0[1] + e0[2] + e0[3]);
}

/* Batch of exchange trials, evaluated independently against the state at
 * batch start.  Candidates d = 0,1,... are drawn in counter order; candidate
 * d is admitted if neither molecule is already in an admitted trial and each
 * of its changed beads is at least r_c (float64 minimum image) from every
 * changed bead of the admitted trials.  Drawing stops after n_trials
 * admissions or draw_cap draws.  Each admitted trial is accepted when
 * u < exp(-dU/kT) (Eq. 1), u from its own Philox block.  Accepted trials are
 * applied and the stored forces refreshed.
 * Outputs per admitted trial t: d[t], X[t], Y[t], du[t], u[t], acc[t].
 * Returns the number admitted. */
int o_swap_batch(osys* s, int n_trials, int draw_cap, int* od, int* oX, int* oY,
                 double* odu, double* ou, int* oacc)
{
    int nadm = 0;
    int* used = (int*)calloc(s->nm, sizeof(int));
    int cap_beads = n_trials * 2 * 64 + 1;
    int* chb = (int*)malloc(sizeof(int) * cap_beads);
    int nchb = 0;
    double rc2 = s->rc * s->rc;
    for (int d = 0; d < draw_cap && nadm < n_trials; ++d) {
        uint32_t w[4];
        draw(s, (uint32_t)d, s->batch, ST_SWAP_DRAW, w);
        int X, Y;
        if (!draw_pair(s, w, &X, &Y)) continue;
        if (used[X] || used[Y]) continue;
        int loc[64];
        int nl = changed_locals(s, s->mkind[X], s->mkind[Y], loc);
        int mine[128], nmine = 0;
        for (int q = 0; q < nl; ++q) mine[nmine++] = s->mfirst[X] + loc[q];
        for (int q = 0; q < nl; ++q) mine[nmine++] = s->mfirst[Y] + loc[q];
        int ok = 1;
        for (int a = 0; a < nmine && ok; ++a)
            for (int b = 0; b < nchb; ++b) {
                double dd[3];
                min_image(s, &s->x[3 * mine[a]], &s->x[3 * chb[b]], dd);
                if (dist2(dd) < rc2) { ok = 0; break; }
            }
        if (!ok) continue;
        used[X] = used[Y] = 1;
        for (int a = 0; a < nmine; ++a) chb[nchb++] = mine[a];
        od[nadm] = d; oX[nadm] = X; oY[nadm] = Y;
        nadm++;
    }
    /* evaluate every admitted trial against the pre-batch state */
    for (int t = 0; t < nadm; ++t) {
        odu[t] = delta_u_pair(s, oX[t], oY[t]);
        uint32_t w[4];
        draw(s, (uint32_t)od[t], s->batch, ST_SWAP_ACCEPT, w);
        ou[t] = u53(w[0], w[1]);
        oacc[t] = ou[t] < exp(-odu[t] / s->kT);
    }
    int any = 0;
    for (int t = 0; t < nadm; ++t)
        if (oacc[t]) {
            int kx = s->mkind[oX[t]];
            s->mkind[oX[t]] = s->mkind[oY[t]];
            s->mkind[oY[t]] = kx;
            any = 1;
        }
    if (any) { force_eval(s, NULL, 0.0, s->f); s->n_fe--; }
    s->n_fe++;     /* one energy evaluation per batch */
    s->batch++;
    free(used); free(chb);
    return nadm;
}

/* ---------------------------------------------------------------- MDAS */
/* One alchemical trajectory (Section 2): select n_pairs disjoint exchange
 * pairs; starting at l=0, K times run M BAOAB steps at fixed l and then raise
 * l by 1/K in one step, adding U_{l+dl}(x) - U_l(x) to the work (Eq. 2); at
 * l=1 accept with probability min(1, exp(-w/kT)) (Eq. 3).  On acceptance
 * the run continues from the l=1 state (kinds exchanged); on rejection the
 * state before the trajectory is restored.  pairs_out gets (X,Y) per pair.
 * Returns the number of pairs selected. */
int o_mdas_cycle(osys* s, int n_pairs, int K, int M, double* w_out, int* acc_out,
                 double* u_out, int* pairs_out)
{
    int* used = (int*)calloc(s->nm, sizeof(int));
    int* mk_b = (int*)malloc(sizeof(int) * s->nm);
    memcpy(mk_b, s->mkind, sizeof(int) * s->nm);
    int np = 0;
    for (int d = 0; d < 64 * n_pairs && np < n_pairs; ++d) {
        uint32_t w[4];
        draw(s, (uint32_t)d, s->cycle, ST_MDAS_SELECT, w);
        int X, Y;
        if (!draw_pair(s, w, &X, &Y)) continue;
        if (used[X] || used[Y]) continue;
        used[X] = used[Y] = 1;
        mk_b[X] = s->mkind[Y]; mk_b[Y] = s->mkind[X];
        if (pairs_out) { pairs_out[2 * np] = X; pairs_out[2 * np + 1] = Y; }
        np++;
    }
    size_t nb = sizeof(double) * 3 * s->n;
    double* x0 = (double*)malloc(nb);
    double* v0 = (double*)malloc(nb);
    double* f0 = (double*)malloc(nb);
    memcpy(x0, s->x, nb); memcpy(v0, s->v, nb); memcpy(f0, s->f, nb);
    double work = 0.0, lam = 0.0;
    if (M == 0) s->n_fe++;   /* the single energy difference of a frozen AT */
    for (int k = 1; k <= K; ++k) {
        for (int m = 0; m < M; ++m) md_one(s, mk_b, lam);
        double lam_new = (double)k / (double)K;
        if (s->mdas_path == 1) {
            work += sc_energy_forces(s, mk_b, lam_new, NULL) - sc_energy_forces(s, mk_b, lam, NULL);
        } else {
            double ea[4], eb[4];
            energy_forces(s, s->mkind, NULL, ea, 1);
            energy_forces(s, mk_b, NULL, eb, 1);
            double ua = ea[0] + ea[1] + ea[2] + ea[3], ub = eb[0] + eb[1] + eb[2] + eb[3];
            double u_new = (1.0 - lam_new) * ua + lam_new * ub;
            double u_old = (1.0 - lam) * ua + lam * ub;
            work += u_new - u_old;
        }
        lam = lam_new;
        if (M > 0) { force_eval(s, mk_b, lam, s->f); s->n_fe--; }
    }
    uint32_t w[4];
    draw(s, 0u, s->cycle, ST_MDAS_ACCEPT, w);
    double u = u53(w[0], w[1]);
    int acc = u < exp(-work / s->kT);
    if (acc) {
        memcpy(s->mkind, mk_b, sizeof(int) * s->nm);
        force_eval(s, NULL, 0.0, s->f); s->n_fe--;
    } else {
        memcpy(s->x, x0, nb); memcpy(s->v, v0, nb); memcpy(s->f, f0, nb);
    }
    s->cycle++;
    if (w_out) *w_out = work;
    if (acc_out) *acc_out = acc;
    if (u_out) *u_out = u;
    free(used); free(mk_b); free(x0); free(v0); free(f0);
    return np;
}

/* U_B - U_A at the current coordinates for the exchange of the given pairs. */
double o_pairs_delta_u(osys* s, int n_pairs, const int* pairs)
{
    int* mk_b = (int*)malloc(sizeof(int) * s->nm);
    memcpy(mk_b, s->mkind, sizeof(int) * s->nm);
    for (int p = 0; p < n_pairs; ++p) {
        int X = pairs[2 * p], Y = pairs[2 * p + 1];
        mk_b[X] = s->mkind[Y]; mk_b[Y] = s->mkind[X];
    }
    double ea[4], eb[4];
    energy_forces(s, s->mkind, NULL, ea, 1);
    energy_forces(s, mk_b, NULL, eb, 1);
    free(mk_b);
    return (eb[0] + eb[1] + eb[2] + eb[3]) - (ea[0] + ea[1] + ea[2] + ea[3]);
}

/* ------------------------------------------------------ mixing observable */
/* Results: mixing is followed through the pair correlation of the PO4
 * beads of one lipid type.  Here: over all unordered pairs of PO4 beads
 * (bead index po4 of the kind) of the molecules of kind `kind` that sit in
 * the same leaflet (leaflet[m] = 0 or 1, -1 skips the molecule), the
 * lateral separation d (x and y, each by the minimum-image convention of
 * the periodic box) falls in bin k when (k w)^2 <= d^2 < ((k+1) w)^2;
 * counts[k] (k < n_bins) gets one per pair.  Plain double loop over pairs. */
static double bin_edge2(int k, double w) { return ((double)k * w) * ((double)k * w); }

void o_pair_histogram(const osys* s, int kind, int po4, const int* leaflet, int n_bins, double w,
                      int64_t* counts)
{
    for (int k = 0; k < n_bins; ++k) counts[k] = 0;
    for (int a = 0; a < s->nm; ++a) {
        if (s->mkind[a] != kind || leaflet[a] < 0) continue;
        const int ia = s->mfirst[a] + po4;
        for (int b = a + 1; b < s->nm; ++b) {
            if (s->mkind[b] != kind || leaflet[b] != leaflet[a]) continue;
            const int ib = s->mfirst[b] + po4;
            double d[3];
            min_image(s, &s->x[3 * ia], &s->x[3 * ib], d);
            const double d2 = d[0] * d[0] + d[1] * d[1];
            int k = (int)(sqrt(d2) / w);
            while (k > 0 && bin_edge2(k, w) > d2) --k;
            while (bin_edge2(k + 1, w) <= d2) ++k;
            if (k < n_bins) counts[k]++;
        }
    }
}
