// runtime.hip -- host side of the membx C-ABI: descriptor checks, arena
// layout, upload, step sequencing, exchange moves, MDAS cycles, queries,
// HIP-graph replay and kernel timing.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "membx.h"
#include "membx_dev.h"

namespace mbx {
// launchers (defined in the kernel translation units)
template <typename R> void launch_rebuild(const Dev<R>&, hipStream_t, bool);
template <typename R> int launch_nonbonded(const Dev<R>&, int, bool, double*, hipStream_t);
template <typename R>
void launch_nonbonded_fused(const Dev<R>&, int, int, R, long long, V4<R>*, V4<R>*, int, hipStream_t);
template <typename R>
void launch_nonbonded_alch(const Dev<R>&, int, R, long long, V4<R>*, V4<R>*, const AlchK<R>&,
                           hipStream_t);
void launch_energy_final(const double*, int, double*, hipStream_t);
template <typename R> void launch_kick_drift(const Dev<R>&, R, long long, int, hipStream_t, int = 0);
template <typename R>
void launch_alch_bridge(const Dev<R>&, const int*, double*, R, R, double, long long, hipStream_t);
template <typename R>
void launch_sc_bridge(const Dev<R>&, const int*, const double*, double*, R, long long, hipStream_t);
template <typename R> void launch_kick(const Dev<R>&, R, long long, hipStream_t);
template <typename R>
int launch_kick_ke(const Dev<R>&, const VrBuf&, R, hipStream_t);
template <typename R>
int launch_nonbonded_kick(const Dev<R>&, int, const VrBuf&, R, hipStream_t);
template <typename R>
void launch_vr_scale(const Dev<R>&, const VrBuf&, int, long long, double, hipStream_t);
template <typename R>
void launch_baro(const Dev<R>&, const double*, double*, double, double, double, double, double,
                 hipStream_t);
template <typename R> void launch_scale_pos(const Dev<R>&, const double*, hipStream_t);
template <typename R> void launch_unscale_vel(const Dev<R>&, const double*, hipStream_t);
template <typename R>
void launch_vr_kick_drift(const Dev<R>&, const VrBuf&, R, long long, int, int, long long, double,
                          hipStream_t, int);
template <typename R> void launch_sd_step(const Dev<R>&, double, double, hipStream_t);
template <typename R> void launch_export(const Dev<R>&, const V4<R>*, double*, hipStream_t);
template <typename R> void launch_import(const Dev<R>&, V4<R>*, const double*, hipStream_t);
void launch_fill_i32(int*, int, size_t, hipStream_t);
template <typename R> void launch_obs_gather(const Dev<R>&, const ObsBuf&, int, int, hipStream_t);
void launch_obs_pairs(const ObsBuf&, int, int, double, double, double, hipStream_t);
void launch_copy(void*, const void*, size_t, hipStream_t);
void launch_add_ctr(long long*, int, long long, hipStream_t);
template <typename R> void launch_select(const Dev<R>&, const Mv&, int, int, int, hipStream_t);
template <typename R> void launch_mark(const Dev<R>&, const Mv&, int, int, hipStream_t);
template <typename R> void launch_du(const Dev<R>&, const Mv&, int, hipStream_t);
template <typename R> void launch_trial_accept(const Dev<R>&, const Mv&, int, hipStream_t);
template <typename R> void launch_du_total(const Dev<R>&, const Mv&, double*, hipStream_t);
template <typename R> void launch_aff_build(const Dev<R>&, const Mv&, int, int, bool, hipStream_t);
template <typename R> void launch_aff_clear(const Dev<R>&, const Mv&, hipStream_t);
template <typename R> void launch_dforce(const Dev<R>&, const Mv&, R, hipStream_t);
template <typename R>
void launch_scforce(const Dev<R>&, const Mv&, double, double, double, hipStream_t, bool = false);
template <typename R>
void launch_scdu(const Dev<R>&, const Mv&, int, double, double, double, hipStream_t);
template <typename R> void launch_dlam(const Dev<R>&, const Mv&, R, hipStream_t);
template <typename R> void launch_commit(const Dev<R>&, const Mv&, int, int, hipStream_t);
template <typename R> void launch_bond_du(const Dev<R>&, const Mv&, double, hipStream_t);
template <typename R> void launch_bond_dforce(const Dev<R>&, const Mv&, double, int, hipStream_t);
template <typename R> void launch_bond_dlam(const Dev<R>&, const Mv&, double, hipStream_t);
template <typename R> void launch_bt_refresh(const Dev<R>&, const Mv&, int, hipStream_t);
void launch_work(double*, double, hipStream_t);
template <typename R> void launch_mdas_accept(const Dev<R>&, const Mv&, hipStream_t);
template <typename R> void launch_snapshot(const Dev<R>&, const Mv&, int, hipStream_t);
template <typename R> void launch_kcnt(const Dev<R>&, const Mv&, int, int, int, hipStream_t);
void launch_set_classes(void* posq, int prec, const int* cls_by_bead, const int* orig, int N,
                        hipStream_t st);
}  // namespace mbx

using namespace mbx;

namespace {

constexpr double KB = 0.00831446261815324;   // kJ/mol/K
constexpr double FELEC = 138.935458;         // kJ mol^-1 nm e^-2
constexpr double BAR = 16.6054;              // bar per kJ mol^-1 nm^-3

struct Status {
    int32_t code;
    std::string msg;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's arena; with base == nullptr it only
// measures.
struct Arena {
    char* base;
    size_t off = 0;
    template <typename T> T* take(size_t n)
    {
        off = align_up(off, 256);
        T* p = base ? (T*)(base + off) : nullptr;
        off += sizeof(T) * (n ? n : 1);
        return p;
    }
};

struct Host {
    // descriptor copies
    int N = 0, nm = 0, nk = 0, nt = 0, prec = 1;
    std::vector<int> kn, kbead_off, kfam, mol_kind0, mol_first, btype;
    std::vector<double> bq, bm;
    std::vector<int> kb_off, kb_n, b_ij, ka_off, ka_n, a_ijk;
    std::vector<double> b_par, a_par;   // (b0,k), (cos0,k)
    std::vector<double> eps, sig;
    double box[3], rc, eps_r, eps_rf, dt, T, gamma;
    uint64_t seed;
    // derived
    std::vector<int> kcls;              // class of each kind bead
    std::vector<std::pair<int, double>> cls;   // (type, charge)
    std::vector<int> excl;              // [N * MAXEXCL]
    std::vector<int> bmols;
    std::vector<int> bt_off;            // per-bead bonded terms (CSR over bead ids)
    std::vector<int> bt;                // 4 ints per entry
    std::vector<double> bt_par;         // 2 per parameter set
    // topology-changing families: per-kind-pair flags, per-kind-bead record
    // templates (4 ints each, MAXBT per kind bead); bt is then MAXBT per bead
    int topo = 0;
    std::vector<int> ktopo, ktpl;
    std::vector<int> sw_list, fam_off, fam_mem, fam_of_kind, chg_n, chg_loc;
    int nfam = 0, maxch = 0, fam_stride = 1;
    // exchange regions (leaflets) and the partner rule (0 anywhere, 1 within
    // X's region, 2 in the other region); members of each family by region
    int xmode = 0;
    std::vector<int> region, reg_off, reg_mem;
    double krf, crf;
    // tuning / capacities
    double skin, skin_max;
    int R, lpb, Kcap, Gcap, T_cap, P_cap;
    // ensemble: 0 Langevin BAOAB; 1 velocity Verlet + stochastic velocity
    // rescaling with coupling time tau_t and the group of each kind
    int ensemble = 0;
    double tau_t = 0.0;
    std::vector<int> kgroup, bmol;      // [nk], [N] molecule of each bead
    double skin_in;   // inner-list buffer delta (nm)
    int prune;        // force passes per inner-list prune; 0: no inner list
    int nc[3], ncell, ne[3], next;   // cell grid at the current skin
    int ncell_cap, next_cap;          // array sizes (grid at the smallest skin)
    int nc_cap[3] = { 0, 0, 0 };      // its cells per axis: the grid never exceeds them
    // pressure coupling every baro_nst MD steps (0: off): P0 (kJ mol^-1 nm^-3),
    // compressibility (its inverse), tau_p (ps)
    int baro_nst = 0;
    double p_ref = 0.0, kappa = 0.0, tau_p = 0.0;
    // 0 stochastic cell rescaling; 1 Parrinello-Rahman with box velocity
    // box_v (nm/ps) and box mass w_box (amu)
    int baro_kind = 0;
    double box_v[3] = { 0.0, 0.0, 0.0 }, w_box = 0.0;
    // MDAS lambda path: 0 linear (Eq. 2), 1 soft-core LJ (Eq. 4), shift (nm^2)
    int mdas_path = 0;
    double sc_delta = 0.05;
    int hnc[3], hcells, mh;
    int aff_cap;
};

// Members of each swap family split by region, ascending molecule ids:
// (family f, region r) occupies reg_mem[reg_off[2 f + r], reg_off[2 f + r + 1]).
static void build_regions(Host& h)
{
    h.reg_off.assign(2 * h.nfam + 1, 0);
    h.reg_mem.clear();
    for (int f = 0; f < h.nfam; ++f)
        for (int r = 0; r < 2; ++r) {
            for (int k = h.fam_off[f]; k < h.fam_off[f + 1]; ++k)
                if (h.region[h.fam_mem[k]] == r) h.reg_mem.push_back(h.fam_mem[k]);
            h.reg_off[2 * f + r + 1] = (int)h.reg_mem.size();
        }
}

// Largest skin the current box allows: cells of edge >= r_cut + skin need at
// least three per axis (the box may have shrunk under pressure coupling).
static double box_skin_limit(const Host& h)
{
    double lim = h.skin_max;
    for (int a = 0; a < 3; ++a) lim = std::min(lim, h.box[a] / 3.0 - h.rc);
    return lim;
}

// Cell grid for list radius r_cut + skin: nc = floor(L / r_list) cells per
// axis (at least 3), plus one halo layer of ghost images.
static void set_grid(Host& h, double skin)
{
    const double rl = h.rc + skin;
    h.ncell = 1;
    for (int a = 0; a < 3; ++a) {
        h.nc[a] = std::max(3, (int)std::floor(h.box[a] / rl));
        if (h.nc_cap[a] > 0) h.nc[a] = std::min(h.nc[a], h.nc_cap[a]);   // box grown: coarser cells
        h.ne[a] = h.nc[a] + 1;
        h.ncell *= h.nc[a];
    }
    h.next = h.ne[0] * h.ne[1] * h.ne[2];
}

Status check_desc(const membx_desc* d, Host& h)
{
    if (!d) return { MEMBX_E_INVAL, "null descriptor" };
    if (d->n_kinds <= 0 || !d->kinds) return { MEMBX_E_INVAL, "no kinds" };
    if (d->n_mols <= 0 || !d->mol_kind) return { MEMBX_E_INVAL, "no molecules" };
    if (!d->pos) return { MEMBX_E_INVAL, "no positions" };
    if (d->n_types <= 0 || d->n_types > 16 || !d->lj_epsilon || !d->lj_sigma)
        return { MEMBX_E_INVAL, "bad LJ tables" };
    if (d->precision != MEMBX_FP64 && d->precision != MEMBX_MIXED)
        return { MEMBX_E_INVAL, "bad precision" };
    if (!(d->r_cut > 0) || !(d->eps_r > 0) || !(d->dt > 0) || !(d->temperature >= 0) ||
        !(d->gamma >= 0))
        return { MEMBX_E_INVAL, "bad physical parameters" };
    h.prec = d->precision;
    h.nk = d->n_kinds;
    h.nt = d->n_types;
    h.kn.resize(h.nk);
    h.kbead_off.resize(h.nk);
    h.kfam.resize(h.nk);
    h.kb_off.resize(h.nk); h.kb_n.resize(h.nk); h.ka_off.resize(h.nk); h.ka_n.resize(h.nk);
    int tot = 0;
    for (int k = 0; k < h.nk; ++k) {
        const membx_kind& K = d->kinds[k];
        if (K.n_beads <= 0 || !K.bead_type || !K.bead_charge || !K.bead_mass)
            return { MEMBX_E_INVAL, "kind " + std::to_string(k) + ": bad beads" };
        h.kn[k] = K.n_beads;
        h.kbead_off[k] = tot;
        tot += K.n_beads;
        h.kfam[k] = K.swap_family;
        for (int b = 0; b < K.n_beads; ++b) {
            if (K.bead_type[b] < 0 || K.bead_type[b] >= h.nt)
                return { MEMBX_E_INVAL, "bead type out of range" };
            if (!(K.bead_mass[b] > 0)) return { MEMBX_E_INVAL, "bead mass must be > 0" };
            h.btype.push_back(K.bead_type[b]);
            h.bq.push_back(K.bead_charge[b]);
            h.bm.push_back(K.bead_mass[b]);
        }
        h.kb_off[k] = (int)h.b_par.size() / 2;
        h.kb_n[k] = K.n_bonds;
        for (int q = 0; q < K.n_bonds; ++q) {
            int i = K.bond_ij[2 * q], j = K.bond_ij[2 * q + 1];
            if (i < 0 || j < 0 || i >= K.n_beads || j >= K.n_beads || i == j)
                return { MEMBX_E_INVAL, "bond index out of range" };
            h.b_ij.push_back(i); h.b_ij.push_back(j);
            h.b_par.push_back(K.bond_b0[q]); h.b_par.push_back(K.bond_k[q]);
        }
        h.ka_off[k] = (int)h.a_par.size() / 2;
        h.ka_n[k] = K.n_angles;
        for (int q = 0; q < K.n_angles; ++q) {
            for (int c = 0; c < 3; ++c) {
                int i = K.angle_ijk[3 * q + c];
                if (i < 0 || i >= K.n_beads) return { MEMBX_E_INVAL, "angle index out of range" };
                h.a_ijk.push_back(i);
            }
            h.a_par.push_back(std::cos(K.angle_theta0[q] * M_PI / 180.0));
            h.a_par.push_back(K.angle_k[q]);
        }
        if ((K.n_bonds > 0 || K.n_angles > 0) && K.n_beads > MAXMB)
            return { MEMBX_E_INVAL, "bonded molecule larger than 16 beads" };
    }
    h.nm = d->n_mols;
    h.mol_kind0.assign(d->mol_kind, d->mol_kind + h.nm);
    h.mol_first.resize(h.nm);
    long long n = 0;
    for (int m = 0; m < h.nm; ++m) {
        int k = h.mol_kind0[m];
        if (k < 0 || k >= h.nk) return { MEMBX_E_INVAL, "molecule kind out of range" };
        h.mol_first[m] = (int)n;
        n += h.kn[k];
    }
    if (n >= (1LL << 27)) return { MEMBX_E_INVAL, "too many beads" };
    h.N = (int)n;
    h.bmol.resize(h.N);
    for (int m = 0; m < h.nm; ++m)
        for (int b = 0; b < h.kn[h.mol_kind0[m]]; ++b) h.bmol[h.mol_first[m] + b] = m;
    h.kgroup.assign(h.nk, 0);
    h.eps.assign(d->lj_epsilon, d->lj_epsilon + h.nt * h.nt);
    h.sig.assign(d->lj_sigma, d->lj_sigma + h.nt * h.nt);
    for (int a = 0; a < 3; ++a) h.box[a] = d->box[a];
    h.rc = d->r_cut; h.eps_r = d->eps_r; h.eps_rf = d->eps_rf;
    h.dt = d->dt; h.T = d->temperature; h.gamma = d->gamma; h.seed = d->seed;
    if (h.prec == MEMBX_MIXED)
        for (int a = 0; a < 3; ++a) h.box[a] = (double)(float)h.box[a];
    // reaction field (eps_rf beyond the cutoff; <= 0 or inf: conducting)
    bool inf_rf = !(h.eps_rf > 0) || std::isinf(h.eps_rf);
    h.krf = inf_rf ? 1.0 / (2.0 * h.rc * h.rc * h.rc)
                   : (h.eps_rf - h.eps_r) / ((2.0 * h.eps_rf + h.eps_r) * h.rc * h.rc * h.rc);
    h.crf = 1.0 / h.rc + h.krf * h.rc * h.rc;
    // tuning
    h.skin = d->skin > 0 ? d->skin : 0.3;
    if (d->skin_max > 0) h.skin_max = std::max(h.skin, d->skin_max);
    else {
        const double lim = std::min(h.box[0], std::min(h.box[1], h.box[2])) / 3.0 - h.rc;
        h.skin_max = std::max(h.skin, std::min(0.6, lim));
    }
    h.R = d->rebuild_interval > 0 ? d->rebuild_interval : 5;
    h.lpb = d->lanes_per_bead > 0 ? d->lanes_per_bead : 8;
    h.prune = d->prune_interval > 1 ? d->prune_interval : 0;
    h.skin_in = h.prune ? std::min(d->skin_inner > 0 ? d->skin_inner : 0.5 * h.skin, h.skin) : 0.0;
    if (h.prune && h.lpb < 2) return { MEMBX_E_INVAL, "an inner list needs lanes_per_bead >= 2" };
    if (h.lpb != 1 && h.lpb != 2 && h.lpb != 4 && h.lpb != 8)
        return { MEMBX_E_INVAL, "lanes_per_bead must be 1, 2, 4 or 8" };
    h.T_cap = d->max_trials > 0 ? d->max_trials : 256;
    h.P_cap = d->max_pairs > 0 ? d->max_pairs : 64;
    if (h.T_cap > 16384 || h.P_cap > 16384) return { MEMBX_E_INVAL, "max_trials/max_pairs > 16384" };
    double rl = h.rc + h.skin_max;
    for (int a = 0; a < 3; ++a)
        if (!(h.box[a] >= 3.0 * rl)) return { MEMBX_E_INVAL, "box must be >= 3 (r_cut + skin)" };
    // arrays hold the finest grid the tuner may choose (skin 0.1 nm)
    set_grid(h, std::min(h.skin, 0.1));
    h.ncell_cap = h.ncell;
    h.next_cap = h.next;
    for (int a = 0; a < 3; ++a) h.nc_cap[a] = h.nc[a];
    set_grid(h, h.skin_max);
    double vol = h.box[0] * h.box[1] * h.box[2];
    double rho = h.N / vol;
    // a multiple of 8: the list is tiled in rows of 64 / lanes_per_bead beads
    if (d->list_capacity > 0) h.Kcap = (d->list_capacity + 7) / 8 * 8;
    else {
        double exp_n = rho * 4.0 / 3.0 * M_PI * rl * rl * rl;
        h.Kcap = (int)std::ceil((exp_n * 1.8 + 24) / 8.0) * 8;
    }
    h.Kcap = std::max(h.Kcap, 96);   // the pair kernel reads the first 96 entries unconditionally
    if (h.Kcap > 512) return { MEMBX_E_INVAL, "list capacity above 512 per bead (lower skin or density)" };
    double gfrac = (1.0 + 1.0 / h.nc[0]) * (1.0 + 1.0 / h.nc[1]) * (1.0 + 1.0 / h.nc[2]) - 1.0;
    h.Gcap = (int)(h.N * gfrac * 1.6) + 4096;
    // list entries hold slots below 2^29, and the force pass addresses the
    // coordinates of a slot by a 32-bit byte offset (32 bytes per slot)
    if ((long long)h.N + h.Gcap >= (1LL << 27))
        return { MEMBX_E_INVAL, "too many beads (beads plus periodic images >= 2^27)" };
    set_grid(h, h.skin);
    // exchange hash (cells >= r_cut)
    h.hcells = 1;
    for (int a = 0; a < 3; ++a) {
        h.hnc[a] = std::max(3, (int)std::floor(h.box[a] / h.rc));
        h.hcells *= h.hnc[a];
    }
    h.mh = 4096;
    return { MEMBX_OK, "" };
}

// Bonded records at MAXBT per bead (bt_off[b] = b MAXBT), rewritten from
// the kind templates for the given molecule kinds (topology-changing
// families: a molecule's records follow its current kind).
static void bt_from_kinds(Host& h, const std::vector<int>& kinds)
{
    h.bt.assign((size_t)h.N * MAXBT * 4, 0);
    h.bt_off.assign(h.N + 1, 0);
    for (int b = 0; b <= h.N; ++b) h.bt_off[b] = b * MAXBT;
    for (int m = 0; m < h.nm; ++m) {
        const int k = kinds[m], f0 = h.mol_first[m];
        for (int l = 0; l < h.kn[k]; ++l)
            for (int t = 0; t < MAXBT; ++t) {
                const int* tp = &h.ktpl[((size_t)(h.kbead_off[k] + l) * MAXBT + t) * 4];
                int* r = &h.bt[((size_t)(f0 + l) * MAXBT + t) * 4];
                const bool on = tp[0] >= 0;
                r[0] = on ? tp[0] : -1;
                r[1] = on ? f0 + tp[1] : f0 + l;
                r[2] = on && tp[2] >= 0 ? f0 + tp[2] : -1;
                r[3] = on ? tp[3] : 0;
            }
    }
}

Status derive(const membx_desc* d, Host& h)
{
    // classes: distinct (type, charge) pairs over all kinds
    h.kcls.resize(h.btype.size());
    for (size_t b = 0; b < h.btype.size(); ++b) {
        auto key = std::make_pair(h.btype[b], h.bq[b]);
        int c = -1;
        for (size_t q = 0; q < h.cls.size(); ++q)
            if (h.cls[q].first == key.first && h.cls[q].second == key.second) c = (int)q;
        if (c < 0) {
            c = (int)h.cls.size();
            h.cls.push_back(key);
        }
        h.kcls[b] = c;
    }
    if ((int)h.cls.size() > MAXCLS) return { MEMBX_E_INVAL, "more than 16 (type, charge) classes" };
    // exclusions: beads joined by a bond (nrexcl = 1)
    h.excl.assign((size_t)h.N * MAXEXCL, -1);
    std::vector<int> nex(h.N, 0);
    // (a molecule of a swap family excludes the pairs bonded in any kind of
    // the family, so that its nonbonded pairs do not depend on its kind)
    for (int m = 0; m < h.nm; ++m) {
        int k0 = h.mol_kind0[m], f0 = h.mol_first[m];
        if (h.kb_n[k0] > 0 || h.ka_n[k0] > 0) h.bmols.push_back(m);
        for (int k = 0; k < h.nk; ++k) {
          if (k != k0 && (h.kfam[k0] < 0 || h.kfam[k] != h.kfam[k0] || h.kn[k] != h.kn[k0])) continue;
          for (int q = 0; q < h.kb_n[k]; ++q) {
            int bq = h.kb_off[k] + q;
            int i = f0 + h.b_ij[2 * bq], j = f0 + h.b_ij[2 * bq + 1];
            bool dup = false;
            for (int e = 0; e < nex[i]; ++e) dup |= h.excl[(size_t)i * MAXEXCL + e] == j;
            if (dup) continue;
            if (nex[i] >= MAXEXCL || nex[j] >= MAXEXCL)
                return { MEMBX_E_INVAL, "a bead has more than 8 bonded partners" };
            h.excl[(size_t)i * MAXEXCL + nex[i]++] = j;
            h.excl[(size_t)j * MAXEXCL + nex[j]++] = i;
          }
        }
    }
    // swap families
    h.fam_of_kind.assign(h.nk, -1);
    std::map<int, int> fid;
    for (int k = 0; k < h.nk; ++k)
        if (h.kfam[k] >= 0) {
            if (!fid.count(h.kfam[k])) {
                int f = (int)fid.size();
                fid[h.kfam[k]] = f;
            }
            h.fam_of_kind[k] = fid[h.kfam[k]];
        }
    h.nfam = (int)fid.size();
    // kinds of one family: same number of beads and masses; their bonded
    // terms may differ (a topology-changing exchange, then at most
    // MAXKN_TOPO beads per molecule)
    h.ktopo.assign((size_t)h.nk * h.nk, 0);
    for (int a = 0; a < h.nk; ++a)
        for (int b = 0; b < h.nk; ++b) {
            if (h.fam_of_kind[a] < 0 || h.fam_of_kind[a] != h.fam_of_kind[b] || a >= b) continue;
            if (h.kn[a] != h.kn[b])
                return { MEMBX_E_INVAL, "kinds of one swap family differ in their number of beads" };
            for (int q = 0; q < h.kn[a]; ++q)
                if (h.bm[h.kbead_off[a] + q] != h.bm[h.kbead_off[b] + q])
                    return { MEMBX_E_INVAL, "kinds of one swap family differ in masses" };
            bool dif = h.kb_n[a] != h.kb_n[b] || h.ka_n[a] != h.ka_n[b];
            for (int q = 0; !dif && q < h.kb_n[a]; ++q)
                for (int c = 0; c < 2; ++c)
                    dif |= h.b_ij[2 * (h.kb_off[a] + q) + c] != h.b_ij[2 * (h.kb_off[b] + q) + c] ||
                           h.b_par[2 * (h.kb_off[a] + q) + c] != h.b_par[2 * (h.kb_off[b] + q) + c];
            for (int q = 0; !dif && q < h.ka_n[a]; ++q) {
                for (int c = 0; c < 3; ++c)
                    dif |= h.a_ijk[3 * (h.ka_off[a] + q) + c] != h.a_ijk[3 * (h.ka_off[b] + q) + c];
                for (int c = 0; c < 2; ++c)
                    dif |= h.a_par[2 * (h.ka_off[a] + q) + c] != h.a_par[2 * (h.ka_off[b] + q) + c];
            }
            if (dif) {
                if (h.kn[a] > MAXKN_TOPO)
                    return { MEMBX_E_INVAL, "a topology-changing swap family has more than 16 beads per molecule" };
                h.ktopo[(size_t)a * h.nk + b] = h.ktopo[(size_t)b * h.nk + a] = 1;
                h.topo = 1;
            }
        }
    h.fam_off.assign(h.nfam + 1, 0);
    std::vector<std::vector<int>> mem(h.nfam);
    for (int m = 0; m < h.nm; ++m) {
        int f = h.fam_of_kind[h.mol_kind0[m]];
        if (f >= 0) { mem[f].push_back(m); h.sw_list.push_back(m); }
    }
    int mx = 0;
    for (int f = 0; f < h.nfam; ++f) {
        h.fam_off[f + 1] = h.fam_off[f] + (int)mem[f].size();
        h.fam_mem.insert(h.fam_mem.end(), mem[f].begin(), mem[f].end());
        mx = std::max(mx, (int)mem[f].size());
    }
    h.fam_stride = mx + 1;
    h.region.assign(h.nm, 0);
    build_regions(h);
    h.chg_n.assign(h.nk * h.nk, 0);
    h.chg_loc.assign(h.nk * h.nk * MAXCH, 0);
    h.maxch = 1;
    for (int a = 0; a < h.nk; ++a)
        for (int b = 0; b < h.nk; ++b) {
            if (a == b || h.fam_of_kind[a] < 0 || h.fam_of_kind[a] != h.fam_of_kind[b]) continue;
            int c = 0;
            for (int q = 0; q < h.kn[a]; ++q)
                if (h.kcls[h.kbead_off[a] + q] != h.kcls[h.kbead_off[b] + q]) {
                    if (c >= MAXCH) return { MEMBX_E_INVAL, "an exchange changes more than 8 beads" };
                    h.chg_loc[(a * h.nk + b) * MAXCH + c++] = q;
                }
            h.chg_n[a * h.nk + b] = c;
            h.maxch = std::max(h.maxch, c);
        }
    // bonded terms as seen from each bead: bonds (role 0 owns the energy,
    // role 1 the partner), angle ends (role 2) and vertices (role 3, owner)
    {
        std::vector<std::vector<std::array<int, 4>>> per(h.N);
        int nbp = (int)h.b_par.size() / 2;
        for (int q = 0; q < nbp; ++q) { h.bt_par.push_back(h.b_par[2 * q]); h.bt_par.push_back(h.b_par[2 * q + 1]); }
        for (size_t q = 0; q < h.a_par.size() / 2; ++q) { h.bt_par.push_back(h.a_par[2 * q]); h.bt_par.push_back(h.a_par[2 * q + 1]); }
        for (int m = 0; m < h.nm; ++m) {
            int k = h.mol_kind0[m], f0 = h.mol_first[m];
            for (int q = 0; q < h.kb_n[k]; ++q) {
                int bq = h.kb_off[k] + q;
                int i = f0 + h.b_ij[2 * bq], j = f0 + h.b_ij[2 * bq + 1];
                per[i].push_back({ 0, j, -1, bq });
                per[j].push_back({ 1, i, -1, bq });
            }
            for (int q = 0; q < h.ka_n[k]; ++q) {
                int aq = h.ka_off[k] + q;
                int i = f0 + h.a_ijk[3 * aq], j = f0 + h.a_ijk[3 * aq + 1], l = f0 + h.a_ijk[3 * aq + 2];
                per[i].push_back({ 2, j, l, nbp + aq });
                per[l].push_back({ 2, j, i, nbp + aq });
                per[j].push_back({ 3, i, l, nbp + aq });
            }
        }
        h.bt_off.assign(h.N + 1, 0);
        for (int b = 0; b < h.N; ++b) {
            if ((int)per[b].size() > MAXBT)
                return { MEMBX_E_INVAL, "a bead takes part in more than 8 bonded terms" };
            h.bt_off[b + 1] = h.bt_off[b] + (int)per[b].size();
            for (auto& e : per[b]) h.bt.insert(h.bt.end(), e.begin(), e.end());
        }
        if (h.bt.empty()) h.bt.assign(4, 0);
        if (h.bt_par.empty()) h.bt_par.assign(2, 0.0);
        // per-kind templates in local bead indices (same construction)
        const int nkb = (int)h.btype.size();
        h.ktpl.assign((size_t)std::max(nkb, 1) * MAXBT * 4, 0);
        std::vector<int> cnt(std::max(nkb, 1), 0);
        auto put = [&](int k, int l, int role, int p1, int p2, int par) -> bool {
            const int kb = h.kbead_off[k] + l;
            if (cnt[kb] >= MAXBT) return false;
            int* r = &h.ktpl[((size_t)kb * MAXBT + cnt[kb]++) * 4];
            r[0] = role; r[1] = p1; r[2] = p2; r[3] = par;
            return true;
        };
        bool ok = true;
        for (int k = 0; k < h.nk; ++k) {
            for (int q = 0; q < h.kb_n[k]; ++q) {
                int bq = h.kb_off[k] + q, i = h.b_ij[2 * bq], j = h.b_ij[2 * bq + 1];
                ok &= put(k, i, 0, j, -1, bq);
                ok &= put(k, j, 1, i, -1, bq);
            }
            for (int q = 0; q < h.ka_n[k]; ++q) {
                int aq = h.ka_off[k] + q;
                int i = h.a_ijk[3 * aq], j = h.a_ijk[3 * aq + 1], l = h.a_ijk[3 * aq + 2];
                ok &= put(k, i, 2, j, l, nbp + aq);
                ok &= put(k, l, 2, j, i, nbp + aq);
                ok &= put(k, j, 3, i, l, nbp + aq);
            }
        }
        if (!ok) return { MEMBX_E_INVAL, "a bead takes part in more than 8 bonded terms" };
        for (int kb = 0; kb < nkb; ++kb)
            for (int t = cnt[kb]; t < MAXBT; ++t) h.ktpl[((size_t)kb * MAXBT + t) * 4] = -1;
        if (h.topo) bt_from_kinds(h, h.mol_kind0);
    }
    h.aff_cap = std::max(h.T_cap, h.P_cap) * 2 * h.maxch * (h.Kcap + 1);
    h.aff_cap = std::min(h.aff_cap, h.N);
    (void)d;
    return { MEMBX_OK, "" };
}

}  // namespace

// ------------------------------------------------------------------- system
struct membx_sys {
    Host h;
    Dev<float> df;
    Dev<double> dd;
    Mv mv;
    hipStream_t st = nullptr, user = nullptr;
    int device = 0;          // device current at creation
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int since = 0;           // steps since the last rebuild
    long long step = 0, batch = 0, cycle = 0, fe = 0, n_rebuilds = 0;
    int nbe_blocks = 0, bd_blocks = 0, ke_blocks = 0;
    double *p_nb = nullptr, *p_bd = nullptr, *p_ke = nullptr;
    double* xbuf = nullptr;  // [3N] export / import buffer
    ObsBuf obs{};            // mixing observable
    VrBuf vr{};              // velocity rescaling thermostat
    int* ibuf = nullptr;     // [N]
    bool graphs = true;
    bool fuse = true;        // force kernel integrates the next step (plain MD)
    int par = 0;             // which coordinate buffer is current (flips per fused step)
    int sp = -1;             // force passes since the last prune; -1: no valid inner list
    std::map<std::tuple<long long, int, int>, hipGraphExec_t> gcache;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
    size_t tev_used = 0;
    long long t_launches = 0;
    double t_ms = 0.0;
    std::string err;
    bool mixed() const { return h.prec == MEMBX_MIXED; }
};

static int32_t fail(membx_sys* s, int32_t code, const std::string& m)
{
    if (s) s->err = m;
    return code;
}

#define HCK(call)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(s, MEMBX_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Prefilter band of the list build around r_list^2: the candidate images are
// stored shifted by +L (rounded, error <= ulp(L)) and r^2 is evaluated in R;
// candidates inside the band are decided by the exact float64 test.
template <typename R>
static void set_list_band(Dev<R>& d, const Host& h)
{
    const double rl = h.rc + h.skin, rl2 = rl * rl;
    const double Lmax = std::max(h.box[0], std::max(h.box[1], h.box[2]));
    const bool f32 = sizeof(R) == 4;
    const double dr = Lmax * (f32 ? std::ldexp(1.0, -22) : std::ldexp(1.0, -51));
    const double margin = rl2 * (f32 ? 4e-6 : 1e-12) + 2.5 * rl * dr;
    d.rl2_lo = (R)(rl2 - margin);
    d.rl2_hi = (R)(rl2 + margin);
    const double rin = h.rc + h.skin_in;
    d.rin2 = h.prune ? (R)(rin * rin) : (R)0;
    d.in_half2 = (R)(0.25 * h.skin_in * h.skin_in);
}

// O part of BAOAB: v <- c1 v + c2 sqrt(kT/m) xi; off (c1 = 1, c2 = 0) under
// the velocity rescaling thermostat, which leaves velocity Verlet
template <typename R>
static void set_friction(Dev<R>& d, const Host& h)
{
    const double c1 = h.ensemble == 1 ? 1.0 : std::exp(-h.gamma * h.dt);
    d.c1 = (R)c1;
    d.c2 = (R)(h.ensemble == 1 ? 0.0 : std::sqrt(1.0 - c1 * c1));
}

template <typename R>
static size_t layout(membx_sys* s, Dev<R>& d, Mv& m, char* base)
{
    Host& h = s->h;
    Arena a{ base };
    int N = h.N;
    int Npad = (N + 63) / 64 * 64;
    d.N = N; d.Npad = Npad; d.nm = h.nm; d.nk = h.nk; d.ncls = (int)h.cls.size();
    d.Kcap = h.Kcap; d.Gcap = h.Gcap; d.nbm = (int)h.bmols.size();
    d.lpb = h.lpb;
    d.lpb_shift = h.lpb == 1 ? 0 : h.lpb == 2 ? 1 : h.lpb == 4 ? 2 : 3;
    d.bg_shift = 6 - d.lpb_shift;
    d.posq = a.take<V4<R>>(N + h.Gcap);
    d.posq_alt = a.take<V4<R>>(N + h.Gcap);
    d.vel = a.take<V4<R>>(N);
    d.frc = a.take<V4<R>>(N);
    d.xref = a.take<V4<R>>(N);
    d.dfrc = a.take<V4<R>>(N);
    d.orig = a.take<int>(N); d.inv = a.take<int>(N); d.alch = a.take<int>(N);
    d.posq_t = a.take<V4<R>>(N); d.vel_t = a.take<V4<R>>(N); d.frc_t = a.take<V4<R>>(N);
    d.orig_t = a.take<int>(N); d.alch_t = a.take<int>(N); d.cell_t = a.take<int>(N);
    d.cell_pos = a.take<int>(N);
    d.cell_cnt = a.take<int>(h.ncell_cap);
    d.cell_start = a.take<int>(h.ncell_cap + 1);
    d.ext_start = a.take<int>(h.next_cap); d.ext_cnt = a.take<int>(h.next_cap);
    d.ext_scan = a.take<int>(2 * h.next_cap + 2);
    d.ghost_owner = a.take<int>(h.Gcap);
    d.n_ghost = a.take<int>(1);
    d.glist = a.take<int>(8 * (size_t)N);
    d.orig_ext = a.take<int>(N + h.Gcap);
    d.bslot = a.take<int4>((size_t)N * MAXBT);
    d.dmax_part = a.take<float>(((size_t)N * 8 + WG - 1) / WG);
    d.nbr = a.take<int>((size_t)h.Kcap * Npad);
    d.ncnt = a.take<int>(N); d.nseg0 = a.take<int>(N);
    d.nbr_in = a.take<int>((size_t)h.Kcap * Npad);
    d.ncnt_in = a.take<int>((size_t)N * 8);
    d.xref_in = a.take<V4<R>>(N);
    d.excl = a.take<int>((size_t)N * MAXEXCL);
    d.exmask = a.take<unsigned>(N);
    d.mol_first = a.take<int>(h.nm); d.mol_kind = a.take<int>(h.nm);
    d.bmols = a.take<int>(h.bmols.size());
    d.kn = a.take<int>(h.nk); d.kbead_off = a.take<int>(h.nk);
    d.kcls = a.take<int>(h.kcls.size());
    d.kb_off = a.take<int>(h.nk); d.kb_n = a.take<int>(h.nk);
    d.b_ij = a.take<int>(h.b_ij.size()); d.b_par = a.take<R>(h.b_par.size());
    d.ka_off = a.take<int>(h.nk); d.ka_n = a.take<int>(h.nk);
    d.a_ijk = a.take<int>(h.a_ijk.size()); d.a_par = a.take<R>(h.a_par.size());
    d.bt_off = a.take<int>(h.bt_off.size());
    d.bt = a.take<int4>(h.bt.size() / 4);
    d.bt_par = a.take<R>(h.bt_par.size());
    d.topo = h.topo;
    d.ktopo = a.take<int>((size_t)h.nk * h.nk);
    d.ktpl = a.take<int4>(h.ktpl.size() / 4);
    d.tabF = a.take<V4<R>>(MAXCLS * MAXCLS); d.tabE = a.take<V4<R>>(MAXCLS * MAXCLS);
    d.flags = a.take<int>(NFLAGS);
    d.ctr = a.take<long long>(NCTR);
    s->nbe_blocks = (N * 8 + WG - 1) / WG;
    s->bd_blocks = ((int)h.bmols.size() + 63) / 64;
    s->ke_blocks = (8 * N + WG - 1) / WG;   // blocks of a force pass at 8 lanes per bead
    d.red = a.take<double>(16 * (size_t)s->nbe_blocks);
    d.eout = a.take<double>(16);
    s->xbuf = a.take<double>(3 * (size_t)N);
    s->obs.leaf = a.take<int>(h.nm);
    s->obs.xy = a.take<double2>(h.nm);
    s->obs.lf = a.take<int>(h.nm);
    s->obs.n = a.take<int>(1);
    s->obs.edge2 = a.take<double>(OBS_MAXBINS + 1);
    s->obs.hist = a.take<unsigned long long>(OBS_MAXBINS);
    s->ibuf = a.take<int>(N);
    s->vr.bmol = a.take<int>(N);
    s->vr.kgroup = a.take<int>(h.nk);
    s->vr.part = a.take<double>(4 * (size_t)s->ke_blocks);
    s->vr.alpha = a.take<double>(2);
    // moves
    int MC = 2 * h.maxch, T = std::max(h.T_cap, h.P_cap);
    m.n_sw = (int)h.sw_list.size();
    m.sw_list = a.take<int>(h.sw_list.size());
    m.fam_of_kind = a.take<int>(h.nk);
    m.fam_off = a.take<int>(h.nfam + 1);
    m.fam_mem = a.take<int>(h.fam_mem.size());
    m.fam_stride = h.fam_stride;
    m.kcnt = a.take<int>((size_t)h.nk * h.fam_stride);
    m.others = a.take<int>((size_t)h.nk * h.fam_stride);
    m.xmode = h.xmode;
    m.region = a.take<int>(h.nm);
    m.reg_off = a.take<int>(h.reg_off.size());
    m.reg_mem = a.take<int>(h.reg_mem.size());
    m.kcnt_r = a.take<int>((size_t)h.nk * 2 * h.fam_stride);
    m.others_r = a.take<int>((size_t)h.nk * 2 * h.fam_stride);
    m.chg_n = a.take<int>(h.nk * h.nk);
    m.chg_loc = a.take<int>(h.nk * h.nk * MAXCH);
    m.maxcht = MC;
    m.c_x = a.take<int>(SEL_CMAX); m.c_y = a.take<int>(SEL_CMAX); m.c_nb = a.take<int>(SEL_CMAX);
    m.c_flag = a.take<int>(SEL_CMAX); m.c_conf_n = a.take<int>(SEL_CMAX);
    m.c_bead = a.take<int>((size_t)SEL_CMAX * MC); m.c_cls = a.take<int>((size_t)SEL_CMAX * MC);
    m.c_pos = a.take<double>(3 * (size_t)SEL_CMAX * MC);
    m.c_conf = a.take<int>((size_t)SEL_CMAX * SEL_CAPC);
    for (int k = 0; k < 3; ++k) { m.hnc[k] = h.hnc[k]; m.hinv[k] = h.hnc[k] / h.box[k]; }
    m.hcells = h.hcells;
    {
        auto pow2 = [](size_t n) { size_t p = 1; while (p < n) p <<= 1; return p; };
        const size_t hb = pow2(2 * (size_t)SEL_CMAX * MC), ab = pow2(2 * (size_t)T * MC),
                     mb = pow2(4 * (size_t)SEL_CMAX);
        m.hb_mask = (int)hb - 1;
        m.hb_word = a.take<unsigned long long>(hb);
        m.hb_ent = a.take<int>(hb * HBW);
        m.ab_mask = (int)ab - 1;
        m.ab_word = a.take<unsigned long long>(ab);
        m.ab_ent = a.take<int>(ab * HBW);
        m.mb_mask = (int)mb - 1;
        m.mb_word = a.take<unsigned long long>(mb);
        m.mb_ent = a.take<int>(mb * HBW);
    }
    m.sel = a.take<int>(SEL_NSEL);
    m.used = a.take<int>(h.nm);
    m.T = T;
    m.r_n = a.take<int>(4);
    m.r_draw = a.take<int>(T); m.r_x = a.take<int>(T); m.r_y = a.take<int>(T);
    m.r_acc = a.take<int>(T);
    m.r_du = a.take<double>(T); m.r_u = a.take<double>(T);
    m.r_nb = a.take<int>(T); m.r_bead = a.take<int>(T * MC); m.r_cls = a.take<int>(T * MC);
    m.r_pos = a.take<double>(3 * (size_t)T * MC);
    m.du_bead = a.take<double>(T * MC);
    m.du_bond = a.take<double>(T);
    m.dfb = a.take<double>((size_t)2 * T * MAXKN_TOPO * 3);
    m.aff_flag = a.take<int>(N);
    m.aff_cap = h.aff_cap;
    m.aff_list = a.take<int>(h.aff_cap);
    m.aff_n = a.take<int>(1);
    m.md = a.take<double>(8);
    m.dsc = a.take<double>((size_t)4 * N);
    m.snap_posq = a.take<V4<R>>(N);
    m.snap_vel = a.take<V4<R>>(N);
    m.snap_frc = a.take<V4<R>>(N);
    m.snap_orig = a.take<int>(N);
    // scalars
    for (int k = 0; k < 3; ++k) {
        d.L[k] = (R)h.box[k]; d.halfL[k] = (R)(0.5 * h.box[k]); d.Ld[k] = h.box[k];
        d.nc[k] = h.nc[k]; d.ne[k] = h.ne[k];
        d.inv_edge[k] = (R)(h.nc[k] / h.box[k]);
    }
    d.ncell = h.ncell; d.next = h.next;
    d.rc2 = (R)(h.rc * h.rc); d.krf = (R)h.krf; d.crf = (R)h.crf;
    d.rc2d = h.rc * h.rc;
    double rl = h.rc + h.skin;
    d.rl2d = rl * rl;
    set_list_band(d, h);
    d.skin_half2 = (R)(0.25 * h.skin * h.skin);
    d.dt = (R)h.dt; d.half_dt = (R)(0.5 * h.dt);
    set_friction(d, h);
    d.kT = (R)(KB * h.T); d.kTd = KB * h.T;
    d.seed = h.seed;
    return a.off + 256;
}

template <typename R> static Dev<R>& dev(membx_sys* s);
template <> Dev<float>& dev<float>(membx_sys* s) { return s->df; }
template <> Dev<double>& dev<double>(membx_sys* s) { return s->dd; }

// ----------------------------------------------------------------- sequences
template <typename R>
static void rebuild(membx_sys* s, bool binned = false)
{
    Dev<R>& d = dev<R>(s);
    launch_rebuild<R>(d, s->st, binned);
    s->since = 0;
    s->n_rebuilds++;
    s->sp = -1;   // slots reordered: the inner list must be rebuilt
}

// nonbonded + bonded forces at the current coordinates (ghosts refreshed
// unless a rebuild just placed them); timed when kernel timing is on
template <typename R>
static void forces(membx_sys* s, bool rebuilt)
{
    Dev<R>& d = dev<R>(s);
    (void)rebuilt;   // the integrator and the rebuild keep the ghost images current
    if (s->timing) {
        if (s->tev_used >= s->tev.size()) {
            hipEvent_t a, b;
            (void)hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
            (void)hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
            s->tev.push_back({ a, b });
        }
        auto& pr = s->tev[s->tev_used++];
        (void)hipEventRecord(pr.first, s->st);
        launch_nonbonded<R>(d, s->h.lpb, false, nullptr, s->st);
        (void)hipEventRecord(pr.second, s->st);
    } else {
        launch_nonbonded<R>(d, s->h.lpb, false, nullptr, s->st);
    }
}

// Exchange the current and the other coordinate buffer.
template <typename R>
static void swap_coords(membx_sys* s)
{
    Dev<R>& d = dev<R>(s);
    std::swap(d.posq, d.posq_alt);
    s->par ^= 1;
}

struct Alch {
    double lam;
    // Langevin segments of a cycle chained by k_alch_bridge: the segment's
    // step counters start at base (the closing kicks of earlier segments did
    // not advance the step counter), its opening update ran in the bridge
    // (open = false) and its closing half-kick runs there too (close = false)
    long long base = 0;
    bool open = true, close = true;
    // the segment's last force pass also makes the boundary to the next
    // segment (lambda + dl), in place of k_alch_bridge (k_nb, FUSE 3)
    bool fuse_next = false;
    double dl = 0.0;
};

template <typename R>
static void alch_terms(membx_sys* s, bool rebuilt, double lam)
{
    Dev<R>& d = dev<R>(s);
    Mv& m = s->mv;
    int T = m.T;
    if (rebuilt) {   // the affected set follows the new slot order
        launch_aff_clear<R>(d, m, s->st);
        launch_aff_build<R>(d, m, 0, T, true, s->st);
    }
    const bool topo = s->h.topo != 0;
    if (s->h.mdas_path == 1) {   // force pass (A) + F_sc(lam) - F_sc(0)
        launch_scforce<R>(d, m, 0.0, lam, s->h.sc_delta, s->st);
        if (topo) launch_bond_dforce<R>(d, m, lam, 0, s->st);   // + lam (F_B - F_A) bonded
        return;
    }
    launch_dforce<R>(d, m, (R)lam, s->st);
    launch_du<R>(d, m, T, s->st);
    if (topo) {
        launch_bond_dforce<R>(d, m, lam, 0, s->st);
        launch_bond_du<R>(d, m, 1.0, s->st);
    }
    launch_du_total<R>(d, m, m.md + 1, s->st);
}

// n steps of BAOAB; alch != nullptr: MDAS segment at fixed lambda.
// launch = false only advances the host mirrors (step bookkeeping, list
// schedule, coordinate buffer) exactly as the launches would.
template <typename R>
static void steps_seq(membx_sys* s, long long n, const Alch* alch, bool launch = true)
{
    Dev<R>& d = dev<R>(s);
    const R h = (R)(0.5 * s->h.dt), full = (R)s->h.dt;
    const bool inner = s->h.prune > 1 && s->h.lpb >= 2;
    // velocity rescaling: every step closes with its own half-kick and the
    // thermostat, so neither kicks nor the next step's update are fused
    const bool vr = s->h.ensemble == 1;
    const double vr_c = vr ? std::exp(-s->h.dt / s->h.tau_t) : 1.0;
    if (alch) s->sp = -1;   // MDAS segments walk the Verlet list; no inner bookkeeping
    bool moved = false;   // the previous force pass already moved the beads
    bool binned = false;  // ... and binned them for the rebuild that follows
    int vr_nblk = 0;      // block partials of the last closing half-kick (its factors pending)
    for (long long k = 0; k < n; ++k) {
        if (!moved && launch) {
            const int chk = (inner && s->sp >= 0) ? 1 : 0;
            // this step rebuilds: the update also bins the new coordinates
            const int bn = s->since + 1 >= s->h.R ? 1 : 0;
            if (vr && k > 0) {
                launch_vr_kick_drift<R>(d, s->vr, h, k, chk, vr_nblk, k - 1, vr_c, s->st, bn);
                binned = bn != 0;
            } else if (!(alch && k == 0 && !alch->open)) {
                launch_kick_drift<R>(d, (k == 0 || vr) ? h : full, (alch ? alch->base : 0) + k, chk,
                                     s->st, bn);
                binned = bn != 0;
            }
        }
        moved = false;
        bool rebuilt = false;
        if (++s->since >= s->h.R) {
            if (launch) rebuild<R>(s, binned);
            else { s->since = 0; s->n_rebuilds++; s->sp = -1; }
            rebuilt = true;
        }
        binned = false;
        if (!alch && !vr && s->fuse && !s->timing && k + 1 < n) {
            // forces of step k and B-A-O-A of step k + 1 in one pass, on the
            // inner list between prunes
            int list = 0;
            if (inner) {
                if (s->sp < 0 || s->sp >= s->h.prune - 1) { list = 2; s->sp = 0; }
                else { list = 1; s->sp++; }
            }
            // the next step rebuilds: this pass also bins the new coordinates
            binned = s->since + 1 >= s->h.R;
            if (launch)
                launch_nonbonded_fused<R>(d, s->h.lpb, list, full, k + 1, d.posq_alt, d.vel,
                                          binned ? 3 : 1, s->st);
            swap_coords<R>(s);
            moved = true;
        } else {
            if (launch) {
                if (vr && !alch && !s->timing) {
                    // forces and the closing half-kick with its block partials in one pass
                    vr_nblk = launch_nonbonded_kick<R>(d, s->h.lpb, s->vr, h, s->st);
                } else if (alch && alch->fuse_next && k + 1 == n) {
                    // the affected beads' F_B - F_A and dU at these coordinates
                    // first (the force update there adds 0), then forces, the
                    // closing half-kick at lambda, the work increment and the
                    // next segment's opening update in one pass
                    alch_terms<R>(s, rebuilt, 0.0);
                    Mv& m = s->mv;
                    const AlchK<R> ak{ m.aff_flag, m.md, (R)alch->lam, (R)alch->dl, alch->dl };
                    launch_nonbonded_alch<R>(d, s->h.lpb, h, alch->base + n, d.posq_alt, d.vel, ak, s->st);
                    swap_coords<R>(s);
                } else {
                    forces<R>(s, rebuilt);
                    if (alch) alch_terms<R>(s, rebuilt, alch->lam);
                    if (vr) vr_nblk = launch_kick_ke<R>(d, s->vr, h, s->st);
                }
            }
            if (s->sp >= 0) s->sp++;
        }
    }
    if (launch) {
        if (vr) {
            if (n > 0) launch_vr_scale<R>(d, s->vr, vr_nblk, n - 1, vr_c, s->st);
            launch_add_ctr(d.ctr, CT_STEP, n, s->st);
        } else {
            if (!alch) launch_kick<R>(d, h, n, s->st);
            else if (alch->close) launch_kick<R>(d, h, alch->base + n, s->st);
        }
    }
}

template <typename R>
static int32_t md_run(membx_sys* s, long long n)
{
    if (n <= 0) return MEMBX_OK;
    const long long chunk = 32;
    while (n > 0) {
        long long k = std::min(n, chunk);
        // graphs hold the box in their kernel arguments: not under pressure coupling
        if (s->graphs && !s->timing && s->h.baro_nst == 0) {
            auto key = std::make_tuple(k, s->since, 2 + s->par + 2 * (s->sp + 1));
            auto it = s->gcache.find(key);
            const int since0 = s->since, par0 = s->par, sp0 = s->sp;
            const long long nrb0 = s->n_rebuilds;
            if (it == s->gcache.end()) {
                hipGraph_t g;
                if (hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return fail(s, MEMBX_E_DEVICE, "stream capture failed");
                steps_seq<R>(s, k, nullptr);
                if (hipStreamEndCapture(s->st, &g) != hipSuccess)
                    return fail(s, MEMBX_E_DEVICE, "stream capture failed");
                hipGraphExec_t ge;
                if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess)
                    return fail(s, MEMBX_E_DEVICE, "graph instantiation failed");
                (void)hipGraphDestroy(g);
                if (s->gcache.size() > 64) {
                    for (auto& kv : s->gcache) (void)hipGraphExecDestroy(kv.second);
                    s->gcache.clear();
                }
                it = s->gcache.emplace(key, ge).first;
                // capture advanced the host mirrors; restore, then replay below
                s->since = since0;
                s->n_rebuilds = nrb0;
                s->sp = sp0;
                if (s->par != par0) swap_coords<R>(s);
            }
            if (hipGraphLaunch(it->second, s->st) != hipSuccess)
                return fail(s, MEMBX_E_DEVICE, "graph launch failed");
            // advance the host mirrors as the sequence does
            steps_seq<R>(s, k, nullptr, false);
        } else {
            steps_seq<R>(s, k, nullptr);
        }
        s->step += k;
        s->fe += k;
        n -= k;
    }
    return MEMBX_OK;
}

template <typename R> static void refresh_forces(membx_sys* s);
template <typename R> static void reset_disp(membx_sys* s);

// Box change to L' = mu L (x, y, z): positions scaled about the origin, the
// cell grid re-planned within the array capacity (cells grow if the box
// does), the box constants of every kernel updated, the list rebuilt and the
// forces refreshed.  E_STATE if an axis fell below three list radii.
template <typename R>
static int32_t rescale_box(membx_sys* s, const double mu[3])
{
    Host& h = s->h;
    Dev<R>& d = dev<R>(s);
    Mv& m = s->mv;
    double nb[3];
    for (int a = 0; a < 3; ++a) nb[a] = h.box[a] * mu[a];
    const double rl = h.rc + h.skin;
    for (int a = 0; a < 3; ++a)
        if (!(nb[a] >= 3.0 * rl)) return fail(s, MEMBX_E_STATE, "box below three list radii");
    launch_scale_pos<R>(d, mu, s->st);
    for (int a = 0; a < 3; ++a) h.box[a] = nb[a];
    set_grid(h, h.skin);
    for (int k = 0; k < 3; ++k) {
        d.L[k] = (R)h.box[k]; d.halfL[k] = (R)(0.5 * h.box[k]); d.Ld[k] = h.box[k];
        d.nc[k] = h.nc[k]; d.ne[k] = h.ne[k];
        d.inv_edge[k] = (R)(h.nc[k] / h.box[k]);
    }
    d.ncell = h.ncell; d.next = h.next;
    set_list_band(d, h);
    h.hcells = 1;
    for (int a = 0; a < 3; ++a) {
        h.hnc[a] = std::max(3, (int)std::floor(h.box[a] / h.rc));
        h.hcells *= h.hnc[a];
        m.hnc[a] = h.hnc[a];
        m.hinv[a] = h.hnc[a] / h.box[a];
    }
    m.hcells = h.hcells;
    HCK(hipMemsetAsync(d.cell_cnt, 0, sizeof(int) * h.ncell_cap, s->st));
    for (auto& kv : s->gcache) (void)hipGraphExecDestroy(kv.second);
    s->gcache.clear();
    refresh_forces<R>(s);
    reset_disp<R>(s);
    return MEMBX_OK;
}

// One pressure coupling at the current state: the energy pass gives the
// virial, k_baro the scale factors (device, from the step counter), the
// host applies them.  Synchronizes.
template <typename R>
static int32_t couple_pressure(membx_sys* s)
{
    Dev<R>& d = dev<R>(s);
    Host& h = s->h;
    const int nnb = launch_nonbonded<R>(d, h.lpb, true, d.red, s->st);
    launch_energy_final(d.red, nnb, d.eout, s->st);
    const double vol = h.box[0] * h.box[1] * h.box[2];
    if (h.baro_kind == 1) {
        // Parrinello-Rahman: the box velocity takes the interval's impulse at
        // the current pressure tensor (x and y: the mean of P_xx and P_yy),
        // the box moves with it; coordinates scale with the box, peculiar
        // velocities against it (host arithmetic in float64)
        double e[13];
        HCK(hipMemcpyAsync(e, d.eout, sizeof(e), hipMemcpyDeviceToHost, s->st));
        HCK(hipStreamSynchronize(s->st));
        const double t = h.baro_nst * h.dt;
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = (e[10 + a] + e[7 + a]) / vol;
        const double pxy = 0.5 * (p[0] + p[1]);
        const double drive[3] = { pxy - h.p_ref, pxy - h.p_ref, p[2] - h.p_ref };
        double mu[3];
        for (int a = 0; a < 3; ++a) {
            h.box_v[a] += t * vol * drive[a] / (h.w_box * h.box[a]);
            mu[a] = (h.box[a] + t * h.box_v[a]) / h.box[a];
        }
        if (!(std::isfinite(mu[0]) && std::isfinite(mu[1]) && std::isfinite(mu[2]) &&
              mu[0] > 0.0 && mu[1] > 0.0 && mu[2] > 0.0))
            return fail(s, MEMBX_E_NONFINITE, "non-finite pressure or box");
        launch_unscale_vel<R>(d, mu, s->st);
        return rescale_box<R>(s, mu);
    }
    launch_baro<R>(d, d.eout, d.eout + 13, h.p_ref, h.kappa, h.tau_p, h.baro_nst * h.dt, vol, s->st);
    double mu[3];
    HCK(hipMemcpyAsync(mu, d.eout + 13, sizeof(mu), hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    if (!(std::isfinite(mu[0]) && std::isfinite(mu[2])))
        return fail(s, MEMBX_E_NONFINITE, "non-finite pressure");
    return rescale_box<R>(s, mu);
}

// n MD steps; under pressure coupling the run stops after every step whose
// index is a multiple of baro_nst to couple
template <typename R>
static int32_t md_steps(membx_sys* s, long long n)
{
    const int nst = s->h.baro_nst;
    if (nst <= 0) return md_run<R>(s, n);
    while (n > 0) {
        const long long k = std::min(n, (long long)(nst - s->step % nst));
        int32_t rc = md_run<R>(s, k);
        if (rc) return rc;
        n -= k;
        if (s->step % nst == 0 && (rc = couple_pressure<R>(s))) return rc;
    }
    return MEMBX_OK;
}

template <typename R>
static void refresh_forces(membx_sys* s)
{
    rebuild<R>(s);
    forces<R>(s, true);
}

template <typename R>
static void kcnt_all(membx_sys* s, bool batch_done = false)
{
    // one work-group per kind (kinds outside every swap family return at once);
    // batch_done: the same launch advances the exchange-batch counter
    launch_kcnt<R>(dev<R>(s), s->mv, 0, s->h.nk, batch_done ? 1 : 0, s->st);
}

template <typename R>
static void swap_seq(membx_sys* s, int n_trials)
{
    Dev<R>& d = dev<R>(s);
    Mv& m = s->mv;
    int T = m.T;
    const bool topo = s->h.topo != 0;
    launch_select<R>(d, m, n_trials, 64 * n_trials, 0, s->st);
    launch_mark<R>(d, m, 0, T, s->st);   // marks only: positions and classes (ghosts too) unchanged
    launch_du<R>(d, m, T, s->st);
    if (topo) launch_bond_du<R>(d, m, 1.0, s->st);   // bonded part of dU
    launch_trial_accept<R>(d, m, T, s->st);   // also clears the rejected trials' marks
    launch_aff_build<R>(d, m, 1, T, false, s->st);
    launch_dforce<R>(d, m, (R)1, s->st);
    if (topo) launch_bond_dforce<R>(d, m, 1.0, 1, s->st);   // accepted: bonded F_new - F_old
    launch_commit<R>(d, m, 0, T, s->st);   // classes of the beads and their images
    if (topo) launch_bt_refresh<R>(d, m, 0, s->st);
    launch_aff_clear<R>(d, m, s->st);
    kcnt_all<R>(s, true);
}

template <typename R>
static int32_t swap_trials(membx_sys* s, int n_trials)
{
    if (s->graphs && !s->timing) {
        auto key = std::make_tuple((long long)n_trials, -1 - s->par, 1);
        auto it = s->gcache.find(key);
        if (it == s->gcache.end()) {
            hipGraph_t g;
            if (hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return fail(s, MEMBX_E_DEVICE, "stream capture failed");
            swap_seq<R>(s, n_trials);
            if (hipStreamEndCapture(s->st, &g) != hipSuccess)
                return fail(s, MEMBX_E_DEVICE, "stream capture failed");
            hipGraphExec_t ge;
            if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess)
                return fail(s, MEMBX_E_DEVICE, "graph instantiation failed");
            (void)hipGraphDestroy(g);
            it = s->gcache.emplace(key, ge).first;
        }
        if (hipGraphLaunch(it->second, s->st) != hipSuccess)
            return fail(s, MEMBX_E_DEVICE, "graph launch failed");
    } else {
        swap_seq<R>(s, n_trials);
    }
    s->batch++;
    s->fe++;
    return MEMBX_OK;
}

template <typename R>
static int32_t mdas(membx_sys* s, int P, int K, int M)
{
    Dev<R>& d = dev<R>(s);
    Mv& m = s->mv;
    int T = m.T;
    hipStream_t st = s->st;
    launch_select<R>(d, m, P, 64 * P, 1, st);
    launch_snapshot<R>(d, m, 0, st);
    launch_mark<R>(d, m, 1, T, st);
    launch_aff_build<R>(d, m, 0, T, false, st);
    launch_fill_i32((int*)m.md, 0, 16, st);
    const bool sc = s->h.mdas_path == 1;
    const bool topo = s->h.topo != 0;
    if (!sc) {
        launch_dforce<R>(d, m, (R)0, st);
        launch_du<R>(d, m, T, st);
        if (topo) {
            launch_bond_dforce<R>(d, m, 0.0, 0, st);
            launch_bond_du<R>(d, m, 1.0, st);
        }
        launch_du_total<R>(d, m, m.md + 1, st);
    } else if (topo) {
        launch_bond_dforce<R>(d, m, 0.0, 0, st);   // F_B - F_A bonded at the start
    }
    // Langevin, linear path: a segment's closing half-kick, the work
    // increment, the move of the forces to the next lambda and the next
    // segment's opening update run as one pass (the same operations)
    const bool bridge = !sc && !topo && M > 0 && s->h.ensemble == 0;
    // ... and that pass is the segment's last force pass (not under kernel timing)
    const bool fbridge = bridge && !s->timing;
    // soft-core path, Langevin: the closing half-kick, the work increment,
    // the affected beads' force update (computed before, held in float64)
    // and the next opening update in one pass (k_sc_bridge)
    const bool scb = sc && !topo && M > 0 && s->h.ensemble == 0;
    long long base = 0;
    double lam = 0.0;
    for (int k = 1; k <= K; ++k) {
        double lam_new = (double)k / (double)K;
        double dl = lam_new - lam;
        if (M > 0) {
            Alch a{ lam };
            if (bridge || scb) {
                a.base = base;
                a.open = k == 1;
                a.close = k == K;
                a.fuse_next = fbridge && k < K;
                a.dl = dl;
            }
            steps_seq<R>(s, M, &a);
            s->step += M;
            s->fe += M;
        }
        if (bridge && k < K) {
            if (!fbridge)
                launch_alch_bridge<R>(d, m.aff_flag, m.md, (R)(0.5 * s->h.dt), (R)dl, dl, base + M, st);
            base += M;
        } else if (scb && k < K) {
            launch_scdu<R>(d, m, T, lam, lam_new, s->h.sc_delta, st);
            launch_du_total<R>(d, m, m.md + 1, st);
            launch_scforce<R>(d, m, lam, lam_new, s->h.sc_delta, st, true);
            launch_sc_bridge<R>(d, m.aff_flag, m.dsc, m.md, (R)(0.5 * s->h.dt), base + M, st);
            base += M;
        } else if (sc) {   // w += U_sc(lam_new) - U_sc(lam) at x; forces follow lambda
            launch_scdu<R>(d, m, T, lam, lam_new, s->h.sc_delta, st);
            if (topo) launch_bond_du<R>(d, m, dl, st);   // bonded terms: linear in lambda
            launch_du_total<R>(d, m, m.md + 1, st);
            launch_work(m.md, 1.0, st);
            launch_scforce<R>(d, m, lam, lam_new, s->h.sc_delta, st);
            if (topo) launch_bond_dlam<R>(d, m, dl, st);
        } else {
            launch_work(m.md, dl, st);
            launch_dlam<R>(d, m, (R)dl, st);
            if (topo) launch_bond_dlam<R>(d, m, dl, st);
        }
        lam = lam_new;
    }
    if (M == 0) s->fe += 1;
    launch_mdas_accept<R>(d, m, st);
    launch_commit<R>(d, m, 1, T, st);
    if (topo) launch_bt_refresh<R>(d, m, 1, st);
    launch_aff_clear<R>(d, m, st);
    launch_snapshot<R>(d, m, 1, st);
    rebuild<R>(s);   // writes the periodic images too
    kcnt_all<R>(s);
    launch_add_ctr(d.ctr, CT_CYCLE, 1, st);
    s->cycle++;
    return MEMBX_OK;
}

// ---------------------------------------------------------------- upload
template <typename R>
static int32_t upload(membx_sys* s, const membx_desc* desc)
{
    Host& h = s->h;
    Dev<R>& d = dev<R>(s);
    Mv& m = s->mv;
    hipStream_t st = s->st;
    std::vector<V4<R>> pos(h.N), vel(h.N);
    std::vector<int> ident(h.N);
    for (int m2 = 0; m2 < h.nm; ++m2) {
        int k = h.mol_kind0[m2];
        for (int b = 0; b < h.kn[k]; ++b) {
            int i = h.mol_first[m2] + b;
            double x[3];
            for (int a = 0; a < 3; ++a) {
                double v = desc->pos[3 * i + a];
                if (!(v >= 0.0 && v < h.box[a])) v -= h.box[a] * std::floor(v / h.box[a]);
                if (!(v < h.box[a])) v = 0.0;
                x[a] = v;
            }
            R xr[3] = { (R)x[0], (R)x[1], (R)x[2] };
            for (int a = 0; a < 3; ++a)
                if (!(xr[a] < (R)h.box[a])) xr[a] = (R)0;
            pos[i] = V4<R>{ xr[0], xr[1], xr[2], (R)0 };
            int c = h.kcls[h.kbead_off[k] + b];
            std::memcpy(&pos[i].w, &c, sizeof(int));
            if (sizeof(R) == 8) {
                long long c64 = (unsigned)c;
                std::memcpy(&pos[i].w, &c64, sizeof(long long));
            }
            double im = 1.0 / h.bm[h.kbead_off[k] + b];
            if (desc->vel)
                vel[i] = V4<R>{ (R)desc->vel[3 * i], (R)desc->vel[3 * i + 1],
                                (R)desc->vel[3 * i + 2], (R)im };
            else
                vel[i] = V4<R>{ 0, 0, 0, (R)im };
            ident[i] = i;
        }
    }
    std::vector<int> minus1(h.N, -1);
    // pair tables
    std::vector<V4<R>> tf(MAXCLS * MAXCLS), te(MAXCLS * MAXCLS);
    int nc = (int)h.cls.size();
    double rc6 = std::pow(h.rc, 6.0), rc12 = rc6 * rc6;
    for (int a = 0; a < nc; ++a)
        for (int b = 0; b < nc; ++b) {
            int ta = h.cls[a].first, tb = h.cls[b].first;
            double e = h.eps[ta * h.nt + tb], sg = h.sig[ta * h.nt + tb];
            double s6 = std::pow(sg, 6.0);
            double c6 = 4.0 * e * s6, c12 = 4.0 * e * s6 * s6;
            double qq = FELEC * h.cls[a].second * h.cls[b].second / h.eps_r;
            tf[a * MAXCLS + b] = V4<R>{ (R)(6.0 * c6), (R)(12.0 * c12), (R)qq,
                                        (R)(2.0 * h.krf * qq) };
            te[a * MAXCLS + b] = V4<R>{ (R)c6, (R)c12, (R)qq, (R)(c12 / rc12 - c6 / rc6) };
        }
    std::vector<R> bpar(h.b_par.begin(), h.b_par.end()), apar(h.a_par.begin(), h.a_par.end());
    std::vector<long long> ctr(NCTR, 0);
    std::vector<int> zeros_flags(NFLAGS, 0);
#define UP(dst, vec)                                                                        \
    if (!(vec).empty())                                                                     \
        HCK(hipMemcpyAsync((dst), (vec).data(), sizeof((vec)[0]) * (vec).size(),           \
                           hipMemcpyHostToDevice, st));
    UP(d.posq, pos);
    UP(d.vel, vel);
    UP(d.orig, ident);
    UP(d.inv, ident);
    UP(d.alch, minus1);
    UP(d.excl, h.excl);
    // bit (j - i + 16): bonded partner j; bit 16: the bead itself
    std::vector<unsigned> exm(h.N, 1u << 16);
    for (int i = 0; i < h.N; ++i)
        for (int e = 0; e < MAXEXCL; ++e) {
            int j = h.excl[(size_t)i * MAXEXCL + e];
            if (j >= 0) exm[i] |= 1u << (j - i + 16);
        }
    UP(d.exmask, exm);
    UP(d.mol_first, h.mol_first);
    UP(d.mol_kind, h.mol_kind0);
    UP(s->vr.bmol, h.bmol);
    UP(s->vr.kgroup, h.kgroup);
    UP(d.bmols, h.bmols);
    UP(d.kn, h.kn);
    UP(d.kbead_off, h.kbead_off);
    UP(d.kcls, h.kcls);
    UP(d.kb_off, h.kb_off);
    UP(d.kb_n, h.kb_n);
    UP(d.b_ij, h.b_ij);
    UP(d.b_par, bpar);
    UP(d.ka_off, h.ka_off);
    UP(d.ka_n, h.ka_n);
    UP(d.a_ijk, h.a_ijk);
    UP(d.a_par, apar);
    std::vector<R> btpar(h.bt_par.begin(), h.bt_par.end());
    UP(d.bt_off, h.bt_off);
    UP(d.bt, h.bt);
    UP(d.bt_par, btpar);
    UP(d.ktopo, h.ktopo);
    UP(d.ktpl, h.ktpl);
    {
        std::vector<double> z((size_t)2 * m.T * MAXKN_TOPO * 3, 0.0);
        HCK(hipMemcpyAsync(m.du_bond, z.data(), sizeof(double) * m.T, hipMemcpyHostToDevice, st));
        HCK(hipMemcpyAsync(m.dfb, z.data(), sizeof(double) * z.size(), hipMemcpyHostToDevice, st));
        HCK(hipStreamSynchronize(st));
    }
    UP(d.tabF, tf);
    UP(d.tabE, te);
    UP(d.flags, zeros_flags);
    UP(d.ctr, ctr);
    UP(m.sw_list, h.sw_list);
    UP(m.fam_of_kind, h.fam_of_kind);
    UP(m.fam_off, h.fam_off);
    UP(m.fam_mem, h.fam_mem);
    UP(m.chg_n, h.chg_n);
    UP(m.chg_loc, h.chg_loc);
    UP(m.region, h.region);
    UP(m.reg_off, h.reg_off);
    UP(m.reg_mem, h.reg_mem);
#undef UP
    HCK(hipMemsetAsync(d.frc, 0, sizeof(V4<R>) * h.N, st));
    // binning counters start at zero; afterwards the cell layout clears them
    // for the next rebuild
    HCK(hipMemsetAsync(d.cell_cnt, 0, sizeof(int) * h.ncell_cap, st));
    HCK(hipMemsetAsync(d.ncnt_in, 0, sizeof(int) * (size_t)h.N * 8, st));
    HCK(hipMemsetAsync(d.dmax_part, 0, sizeof(float) * (((size_t)h.N * 8 + WG - 1) / WG), st));
    HCK(hipMemsetAsync(m.hb_word, 0, sizeof(unsigned long long) * ((size_t)m.hb_mask + 1), st));
    HCK(hipMemsetAsync(m.mb_word, 0, sizeof(unsigned long long) * ((size_t)m.mb_mask + 1), st));
    HCK(hipMemsetAsync(m.ab_word, 0, sizeof(unsigned long long) * ((size_t)m.ab_mask + 1), st));
    HCK(hipMemsetAsync(m.sel, 0, sizeof(int) * SEL_NSEL, st));
    HCK(hipMemsetAsync(m.others, 0, sizeof(int) * (size_t)h.nk * h.fam_stride, st));
    HCK(hipMemsetAsync(m.used, 0, sizeof(int) * h.nm, st));
    HCK(hipMemsetAsync(m.r_n, 0, sizeof(int) * 4, st));
    HCK(hipMemsetAsync(m.aff_flag, 0, sizeof(int) * h.N, st));
    HCK(hipMemsetAsync(m.aff_n, 0, sizeof(int), st));
    HCK(hipMemsetAsync(m.md, 0, sizeof(double) * 8, st));
    HCK(hipMemsetAsync(m.kcnt, 0, sizeof(int) * (size_t)h.nk * h.fam_stride, st));
    HCK(hipMemsetAsync(m.kcnt_r, 0, sizeof(int) * (size_t)h.nk * 2 * h.fam_stride, st));
    HCK(hipMemsetAsync(m.others_r, 0, sizeof(int) * (size_t)h.nk * 2 * h.fam_stride, st));
    kcnt_all<R>(s);
    refresh_forces<R>(s);
    HCK(hipStreamSynchronize(st));   // host staging vectors go out of scope
    HCK(hipGetLastError());
    return MEMBX_OK;
}

// --------------------------------------------------------------- dispatch
#define DISPATCH(s, fn, ...) ((s)->mixed() ? fn<float>(__VA_ARGS__) : fn<double>(__VA_ARGS__))

static int32_t begin(membx_sys* s)
{
    // order the library stream after the caller's stream
    if (hipEventRecord(s->ev_in, s->user) != hipSuccess ||
        hipStreamWaitEvent(s->st, s->ev_in, 0) != hipSuccess)
        return fail(s, MEMBX_E_DEVICE, "stream ordering failed");
    return MEMBX_OK;
}
static int32_t end(membx_sys* s)
{
    if (hipEventRecord(s->ev_out, s->st) != hipSuccess ||
        hipStreamWaitEvent(s->user, s->ev_out, 0) != hipSuccess)
        return fail(s, MEMBX_E_DEVICE, "stream ordering failed");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s, MEMBX_E_DEVICE, hipGetErrorString(e));
    return MEMBX_OK;
}

static int32_t read_flags(membx_sys* s, int* fl)
{
    int* dflags = s->mixed() ? s->df.flags : s->dd.flags;
    if (hipMemcpyAsync(fl, dflags, sizeof(int) * NFLAGS, hipMemcpyDeviceToHost, s->st) != hipSuccess ||
        hipStreamSynchronize(s->st) != hipSuccess)
        return fail(s, MEMBX_E_DEVICE, "flag read failed");
    return MEMBX_OK;
}

static int32_t flag_status(membx_sys* s, const int* fl)
{
    if (fl[FL_LIST_OVF])
        return fail(s, MEMBX_E_LIST_OVERFLOW,
                    "neighbour list capacity exceeded: a bead needed " + std::to_string(fl[FL_LIST_NEED]) +
                    " entries, list_capacity is " + std::to_string(s->h.Kcap) +
                    "; recreate the system with a larger list_capacity (or a smaller skin) and "
                    "restore the last state taken before this error");
    if (fl[FL_GHOST_OVF] || fl[FL_AFF_OVF])
        return fail(s, MEMBX_E_LIST_OVERFLOW, "ghost-image / affected-set capacity exceeded");
    if (fl[FL_SKIN]) return fail(s, MEMBX_E_SKIN, "a bead moved more than skin/2 between rebuilds");
    if (fl[FL_SKIN_IN])
        return fail(s, MEMBX_E_SKIN, "a bead moved more than skin_inner/2 between inner-list prunes");
    return MEMBX_OK;
}

// ================================================================== C-ABI
// (C linkage comes from the declarations in membx.h)

int32_t membx_sys_bytes(const membx_desc* desc, uint64_t* bytes)
{
    membx_sys tmp;
    Status st = check_desc(desc, tmp.h);
    if (st.code) return st.code;
    st = derive(desc, tmp.h);
    if (st.code) return st.code;
    size_t b = tmp.mixed() ? layout<float>(&tmp, tmp.df, tmp.mv, nullptr)
                           : layout<double>(&tmp, tmp.dd, tmp.mv, nullptr);
    if (bytes) *bytes = b;
    return MEMBX_OK;
}

int32_t membx_sys_create(const membx_desc* desc, void* dev_arena, uint64_t arena_bytes,
                         void* hip_stream, membx_sys** out)
{
    if (!out) return MEMBX_E_INVAL;
    *out = nullptr;
    membx_sys* s = new membx_sys();
    Status stt = check_desc(desc, s->h);
    if (!stt.code) stt = derive(desc, s->h);
    if (stt.code) { delete s; return stt.code; }
    size_t need = s->mixed() ? layout<float>(s, s->df, s->mv, nullptr)
                             : layout<double>(s, s->dd, s->mv, nullptr);
    if (!dev_arena || arena_bytes < need) { delete s; return MEMBX_E_NOMEM; }
    char* base = (char*)(((uintptr_t)dev_arena + 255) / 256 * 256);
    if ((uintptr_t)base + need - 256 > (uintptr_t)dev_arena + arena_bytes) { delete s; return MEMBX_E_NOMEM; }
    if (s->mixed()) layout<float>(s, s->df, s->mv, base);
    else layout<double>(s, s->dd, s->mv, base);
    s->user = (hipStream_t)hip_stream;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return MEMBX_E_DEVICE; }
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming) != hipSuccess) {
        delete s;
        return MEMBX_E_DEVICE;
    }
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, upload, s, desc);
    if (!rc) rc = end(s);
    if (rc) { membx_sys_destroy(s); return rc; }
    *out = s;
    return MEMBX_OK;
}

int32_t membx_sys_destroy(membx_sys* s)
{
    if (!s) return MEMBX_OK;
    if (s->st) (void)hipStreamSynchronize(s->st);
    for (auto& kv : s->gcache) (void)hipGraphExecDestroy(kv.second);
    for (auto& pr : s->tev) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    if (s->ev_in) (void)hipEventDestroy(s->ev_in);
    if (s->ev_out) (void)hipEventDestroy(s->ev_out);
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return MEMBX_OK;
}

int32_t membx_md_step(membx_sys* s, int64_t n_steps)
{
    if (!s || n_steps < 0) return fail(s, MEMBX_E_INVAL, "bad arguments");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, md_steps, s, (long long)n_steps);
    if (!rc) rc = end(s);
    return rc;
}

int32_t membx_mc_swap_trials(membx_sys* s, int32_t n_trials, int32_t* n_admitted,
                             int32_t* n_accepted, membx_trial* out)
{
    if (!s) return MEMBX_E_INVAL;
    if (n_trials <= 0 || n_trials > s->h.T_cap)
        return fail(s, MEMBX_E_INVAL, "n_trials must be in [1, max_trials]");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, swap_trials, s, n_trials);
    if (!rc) rc = end(s);
    if (rc) return rc;
    if (n_admitted || n_accepted || out) {
        Mv& m = s->mv;
        int rn[4];
        HCK(hipMemcpyAsync(rn, m.r_n, sizeof(rn), hipMemcpyDeviceToHost, s->st));
        HCK(hipStreamSynchronize(s->st));
        int na = rn[0];
        std::vector<int> dr(na), x(na), y(na), ac(na);
        std::vector<double> du(na), u(na);
        if (na > 0) {
            HCK(hipMemcpyAsync(dr.data(), m.r_draw, sizeof(int) * na, hipMemcpyDeviceToHost, s->st));
            HCK(hipMemcpyAsync(x.data(), m.r_x, sizeof(int) * na, hipMemcpyDeviceToHost, s->st));
            HCK(hipMemcpyAsync(y.data(), m.r_y, sizeof(int) * na, hipMemcpyDeviceToHost, s->st));
            HCK(hipMemcpyAsync(ac.data(), m.r_acc, sizeof(int) * na, hipMemcpyDeviceToHost, s->st));
            HCK(hipMemcpyAsync(du.data(), m.r_du, sizeof(double) * na, hipMemcpyDeviceToHost, s->st));
            HCK(hipMemcpyAsync(u.data(), m.r_u, sizeof(double) * na, hipMemcpyDeviceToHost, s->st));
            HCK(hipStreamSynchronize(s->st));
        }
        int nacc = 0;
        for (int t = 0; t < na; ++t) {
            nacc += ac[t] != 0;
            if (out) out[t] = membx_trial{ dr[t], x[t], y[t], ac[t], du[t], u[t] };
        }
        if (n_admitted) *n_admitted = na;
        if (n_accepted) *n_accepted = nacc;
    }
    return MEMBX_OK;
}

int32_t membx_mdas_cycle(membx_sys* s, int32_t n_pairs, int32_t k_increments, int32_t m_steps,
                         double* work, int32_t* accepted, int32_t* pairs_out)
{
    if (!s) return MEMBX_E_INVAL;
    if (n_pairs <= 0 || n_pairs > s->h.P_cap || k_increments <= 0 || m_steps < 0)
        return fail(s, MEMBX_E_INVAL, "bad MDAS arguments");
    if (s->h.sw_list.empty()) return fail(s, MEMBX_E_STATE, "no exchangeable molecules");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, mdas, s, n_pairs, k_increments, m_steps);
    if (!rc) rc = end(s);
    if (rc) return rc;
    if (work || accepted || pairs_out) {
        double md[8];
        int rn[4];
        HCK(hipMemcpyAsync(md, s->mv.md, sizeof(md), hipMemcpyDeviceToHost, s->st));
        HCK(hipMemcpyAsync(rn, s->mv.r_n, sizeof(rn), hipMemcpyDeviceToHost, s->st));
        HCK(hipStreamSynchronize(s->st));
        if (work) *work = md[0];
        if (accepted) *accepted = md[2] != 0.0;
        if (pairs_out) {
            int np = rn[0];
            std::vector<int> x(np), y(np);
            if (np) {
                HCK(hipMemcpyAsync(x.data(), s->mv.r_x, sizeof(int) * np, hipMemcpyDeviceToHost, s->st));
                HCK(hipMemcpyAsync(y.data(), s->mv.r_y, sizeof(int) * np, hipMemcpyDeviceToHost, s->st));
                HCK(hipStreamSynchronize(s->st));
            }
            for (int p = 0; p < n_pairs; ++p) {
                pairs_out[2 * p] = p < np ? x[p] : -1;
                pairs_out[2 * p + 1] = p < np ? y[p] : -1;
            }
        }
    }
    return MEMBX_OK;
}

// Largest displacement of a bead from its position at the last rebuild seen
// since the last reset of the integrator's per-block maxima (nm).
template <typename R>
static int32_t max_disp(membx_sys* s, double* out)
{
    Dev<R>& d = dev<R>(s);
    const int nb = (int)(((size_t)d.N * 8 + WG - 1) / WG);
    std::vector<float> v(nb);
    HCK(hipMemcpyAsync(v.data(), d.dmax_part, sizeof(float) * nb, hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    float m = 0.f;
    for (float x : v) m = std::max(m, x);
    *out = std::sqrt((double)m);
    return MEMBX_OK;
}

// Zero the skin-violation count and the displacement maxima.
template <typename R>
static void reset_disp(membx_sys* s)
{
    Dev<R>& d = dev<R>(s);
    launch_fill_i32((int*)d.dmax_part, 0, ((size_t)d.N * 8 + WG - 1) / WG, s->st);
    launch_fill_i32(d.flags + FL_SKIN, 0, 1, s->st);
    launch_fill_i32(d.flags + FL_SKIN_IN, 0, 1, s->st);
    launch_fill_i32(d.flags + FL_HIT_OVF, 0, 1, s->st);
}

// Block partials of the energy pass: 16 doubles per work-group it launches.
static size_t energy_partials(const membx_sys* s)
{
    return 16 * (((size_t)s->h.N * s->h.lpb + WG - 1) / WG);
}

// part: the energy pass's block partials (energy_partials(s) doubles), eout:
// their 16 final sums; the arena's buffers unless the caller brings others
template <typename R>
static int32_t energies_impl(membx_sys* s, membx_energy* out, double* part = nullptr,
                             double* eout = nullptr)
{
    Dev<R>& d = dev<R>(s);
    if (!part) part = d.red;
    if (!eout) eout = d.eout;
    int nnb = launch_nonbonded<R>(d, s->h.lpb, true, part, s->st);
    launch_energy_final(part, nnb, eout, s->st);
    double e[16];
    int fl[NFLAGS];
    HCK(hipMemcpyAsync(e, eout, sizeof(double) * 13, hipMemcpyDeviceToHost, s->st));
    int32_t rc = read_flags(s, fl);
    if (rc) return rc;
    membx_energy E{};
    E.lj = e[0]; E.rf = e[1]; E.bond = e[2]; E.angle = e[3]; E.kinetic = e[4];
    E.potential = e[0] + e[1] + e[2] + e[3];
    E.total = E.potential + e[4];
    E.n_pairs_in_cutoff = (int64_t)std::llround(e[5]);
    E.n_list_entries = (int64_t)std::llround(e[6]);
    const double vol = s->h.box[0] * s->h.box[1] * s->h.box[2];
    for (int a = 0; a < 3; ++a) {
        E.virial[a] = e[7 + a];
        E.mv2[a] = e[10 + a];
        E.pressure[a] = (e[10 + a] + e[7 + a]) / vol * BAR;
    }
    E.fe_count = s->fe; E.step = s->step; E.batch = s->batch; E.cycle = s->cycle;
    E.n_rebuilds = s->n_rebuilds;
    E.n_skin_violations = (int64_t)fl[FL_SKIN] + fl[FL_SKIN_IN];
    {
        double dm = 0.0;
        int32_t rc2 = max_disp<R>(s, &dm);
        if (rc2) return rc2;
        E.max_displacement = dm;
    }
    E.list_retests = fl[FL_HIT_OVF] ? 1 : 0;
    if (out) *out = E;
    if (!std::isfinite(E.total)) return fail(s, MEMBX_E_NONFINITE, "non-finite energy");
    return flag_status(s, fl);
}

int32_t membx_energies(membx_sys* s, membx_energy* out)
{
    if (!s) return MEMBX_E_INVAL;
    int32_t rc = begin(s);
    if (rc) return rc;
    rc = DISPATCH(s, energies_impl, s, out);
    int32_t rc2 = end(s);
    return rc ? rc : rc2;
}

// ------------------------------------------------------ allocation-free energies
// Scratch of membx_energies_noalloc: the energy pass's block partials and
// their final sums live in this file-scope device array instead of the
// system's arena.  Each device holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress gives
// on that device (the array's name is a host-side stand-in).
constexpr size_t NOALLOC_DOUBLES = (size_t)1 << 20;   // 8 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
constexpr int NOALLOC_MAXDEV = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[NOALLOC_MAXDEV];

// Address of the scratch array on device dev, looked up once per device
// with that device current.
static int32_t scratch_on(membx_sys* s, int dev, double** out)
{
    if (dev < 0 || dev >= NOALLOC_MAXDEV) return fail(s, MEMBX_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return fail(s, MEMBX_E_DEVICE, "hipGetDevice failed");
        if (cur != dev && hipSetDevice(dev) != hipSuccess)
            return fail(s, MEMBX_E_DEVICE, "hipSetDevice failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(s, MEMBX_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                               hipGetErrorString(e));
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return MEMBX_OK;
}

int32_t membx_energies_noalloc(membx_sys* s, membx_energy* out)
{
    if (!s) return MEMBX_E_INVAL;
    const size_t need = energy_partials(s) + 16;
    if (need > NOALLOC_DOUBLES)
        return fail(s, MEMBX_E_NOMEM, "system too large for the allocation-free energy scratch (" +
                                          std::to_string(need * 8) + " bytes needed, " +
                                          std::to_string(NOALLOC_DOUBLES * 8) + " available)");
    double* sp = nullptr;
    int32_t rc = scratch_on(s, s->device, &sp);
    if (rc) return rc;
    rc = begin(s);
    if (rc) return rc;
    double* part = sp;
    double* eout = sp + energy_partials(s);
    rc = s->mixed() ? energies_impl<float>(s, out, part, eout) : energies_impl<double>(s, out, part, eout);
    int32_t rc2 = end(s);
    return rc ? rc : rc2;
}

template <typename R>
static int32_t get_state_impl(membx_sys* s, double* pos, double* vel, int32_t* mol_kind)
{
    Dev<R>& d = dev<R>(s);
    size_t nb = sizeof(double) * 3 * d.N;
    if (pos) {
        launch_export<R>(d, d.posq, s->xbuf, s->st);
        HCK(hipMemcpyAsync(pos, s->xbuf, nb, hipMemcpyDeviceToHost, s->st));
        HCK(hipStreamSynchronize(s->st));
    }
    if (vel) {
        launch_export<R>(d, d.vel, s->xbuf, s->st);
        HCK(hipMemcpyAsync(vel, s->xbuf, nb, hipMemcpyDeviceToHost, s->st));
        HCK(hipStreamSynchronize(s->st));
    }
    if (mol_kind) {
        HCK(hipMemcpyAsync(mol_kind, d.mol_kind, sizeof(int) * d.nm, hipMemcpyDeviceToHost, s->st));
        HCK(hipStreamSynchronize(s->st));
    }
    return MEMBX_OK;
}

int32_t membx_get_state(membx_sys* s, double* pos, double* vel, int32_t* mol_kind,
                        int64_t* counters)
{
    if (!s) return MEMBX_E_INVAL;
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, get_state_impl, s, pos, vel, mol_kind);
    if (!rc) rc = end(s);
    if (counters) { counters[0] = s->step; counters[1] = s->batch; counters[2] = s->cycle; }
    return rc;
}

template <typename R>
static int32_t set_state_impl(membx_sys* s, const double* pos, const double* vel,
                              const int32_t* mol_kind, const int64_t* counters)
{
    Dev<R>& d = dev<R>(s);
    Host& h = s->h;
    size_t nb = sizeof(double) * 3 * d.N;
    std::vector<double> tmp;
    for (size_t q = 0; q < 3 * (size_t)d.N; ++q)
        if ((pos && !std::isfinite(pos[q])) || (vel && !std::isfinite(vel[q])))
            return fail(s, MEMBX_E_NONFINITE, "non-finite coordinate or velocity (bead " +
                        std::to_string(q / 3) + "); the state is unchanged");
    if (mol_kind)
        for (int m = 0; m < h.nm; ++m) {
            int k = mol_kind[m], k0 = h.mol_kind0[m];
            if (k < 0 || k >= h.nk || h.kn[k] != h.kn[k0] ||
                (k != k0 && (h.fam_of_kind[k] < 0 || h.fam_of_kind[k] != h.fam_of_kind[k0])))
                return fail(s, MEMBX_E_INVAL, "mol_kind must keep each molecule in its family");
        }
    if (counters && (counters[0] < 0 || counters[1] < 0 || counters[2] < 0))
        return fail(s, MEMBX_E_INVAL, "negative counter");
    if (pos) {
        tmp.assign(pos, pos + 3 * (size_t)d.N);
        for (int i = 0; i < d.N; ++i)
            for (int a = 0; a < 3; ++a) {
                double& v = tmp[3 * i + a];
                if (!(v >= 0.0 && v < h.box[a])) {
                    v = std::fmod(v, h.box[a]);          // exact, in (-L, L)
                    if (v < 0.0) v += h.box[a];
                }
                if (!(v >= 0.0 && v < h.box[a])) v = 0.0;   // v + L rounded up to L
            }
        HCK(hipMemcpyAsync(s->xbuf, tmp.data(), nb, hipMemcpyHostToDevice, s->st));
        launch_import<R>(d, d.posq, s->xbuf, s->st);
        HCK(hipStreamSynchronize(s->st));
    }
    if (vel) {
        HCK(hipMemcpyAsync(s->xbuf, vel, nb, hipMemcpyHostToDevice, s->st));
        launch_import<R>(d, d.vel, s->xbuf, s->st);
        HCK(hipStreamSynchronize(s->st));
    }
    std::vector<int> cls;
    if (mol_kind) {
        cls.resize(d.N);
        for (int m = 0; m < h.nm; ++m)
            for (int b = 0; b < h.kn[mol_kind[m]]; ++b)
                cls[h.mol_first[m] + b] = h.kcls[h.kbead_off[mol_kind[m]] + b];
        HCK(hipMemcpyAsync(d.mol_kind, mol_kind, sizeof(int) * d.nm, hipMemcpyHostToDevice, s->st));
        if (h.topo) {   // bonded records follow the molecules' new kinds
            bt_from_kinds(h, std::vector<int>(mol_kind, mol_kind + h.nm));
            HCK(hipMemcpyAsync(d.bt, h.bt.data(), sizeof(int) * h.bt.size(), hipMemcpyHostToDevice, s->st));
        }
        HCK(hipMemcpyAsync(s->ibuf, cls.data(), sizeof(int) * d.N, hipMemcpyHostToDevice, s->st));
        launch_set_classes(d.posq, s->mixed() ? 1 : 0, s->ibuf, d.orig, d.N, s->st);
        kcnt_all<R>(s);
        HCK(hipStreamSynchronize(s->st));
    }
    if (counters) {
        s->step = counters[0]; s->batch = counters[1]; s->cycle = counters[2];
        long long c[NCTR] = { counters[0], counters[1], counters[2], 0 };
        HCK(hipMemcpyAsync(d.ctr, c, sizeof(c), hipMemcpyHostToDevice, s->st));
        HCK(hipStreamSynchronize(s->st));
    }
    refresh_forces<R>(s);
    HCK(hipStreamSynchronize(s->st));
    return MEMBX_OK;
}

int32_t membx_set_state(membx_sys* s, const double* pos, const double* vel,
                        const int32_t* mol_kind, const int64_t* counters)
{
    if (!s) return MEMBX_E_INVAL;
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, set_state_impl, s, pos, vel, mol_kind, counters);
    if (!rc) rc = end(s);
    return rc;
}

template <typename R>
static int32_t forces_impl(membx_sys* s, double* f)
{
    Dev<R>& d = dev<R>(s);
    launch_export<R>(d, d.frc, s->xbuf, s->st);
    HCK(hipMemcpyAsync(f, s->xbuf, sizeof(double) * 3 * d.N, hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    return MEMBX_OK;
}

int32_t membx_forces(membx_sys* s, double* f)
{
    if (!s || !f) return fail(s, MEMBX_E_INVAL, "bad arguments");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, forces_impl, s, f);
    if (!rc) rc = end(s);
    return rc;
}

template <typename R>
static int32_t pairset_impl(membx_sys* s, int32_t* ij, int64_t cap, int64_t* n)
{
    Dev<R>& d = dev<R>(s);
    rebuild<R>(s);
    forces<R>(s, true);
    int N = d.N, G = 0;
    std::vector<int> cnt(N), orig(N), own;
    std::vector<int> nbr((size_t)d.Kcap * d.Npad);
    HCK(hipMemcpyAsync(&G, d.n_ghost, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    own.resize(std::max(G, 1));
    HCK(hipMemcpyAsync(cnt.data(), d.ncnt, sizeof(int) * N, hipMemcpyDeviceToHost, s->st));
    HCK(hipMemcpyAsync(orig.data(), d.orig, sizeof(int) * N, hipMemcpyDeviceToHost, s->st));
    if (G) HCK(hipMemcpyAsync(own.data(), d.ghost_owner, sizeof(int) * G, hipMemcpyDeviceToHost, s->st));
    HCK(hipMemcpyAsync(nbr.data(), d.nbr, sizeof(int) * nbr.size(), hipMemcpyDeviceToHost, s->st));
    int fl[NFLAGS];
    int32_t rc = read_flags(s, fl);
    if (rc) return rc;
    if (fl[FL_LIST_OVF] || fl[FL_GHOST_OVF]) return flag_status(s, fl);
    int64_t k = 0;
    for (int i = 0; i < N; ++i) {
        int oi = orig[i];
        for (int q = 0; q < cnt[i]; ++q) {
            int j = nbr[nbr_index(i, q, d.Kcap, d.lpb)] & JMASK;
            int oj = j < N ? orig[j] : orig[own[j - N]];
            if (oi < oj) {
                if (k < cap) { ij[2 * k] = oi; ij[2 * k + 1] = oj; }
                ++k;
            }
        }
    }
    if (n) *n = k;
    return MEMBX_OK;
}

int32_t membx_pairset_export(membx_sys* s, int32_t* ij, int64_t cap, int64_t* n)
{
    if (!s || (cap > 0 && !ij)) return fail(s, MEMBX_E_INVAL, "bad arguments");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, pairset_impl, s, ij, cap, n);
    if (!rc) rc = end(s);
    return rc;
}

template <typename R>
static int32_t hist_impl(membx_sys* s, int kind, int po4, const int32_t* leaflet, int nb, double w,
                         int64_t* counts)
{
    Dev<R>& d = dev<R>(s);
    Host& h = s->h;
    std::vector<double> e2(nb + 1);
    for (int k = 0; k <= nb; ++k) e2[k] = ((double)k * w) * ((double)k * w);
    HCK(hipMemcpyAsync(s->obs.leaf, leaflet, sizeof(int) * h.nm, hipMemcpyHostToDevice, s->st));
    HCK(hipMemcpyAsync(s->obs.edge2, e2.data(), sizeof(double) * (nb + 1), hipMemcpyHostToDevice, s->st));
    launch_fill_i32(s->obs.n, 0, 1, s->st);
    launch_fill_i32(reinterpret_cast<int*>(s->obs.hist), 0, 2 * (size_t)nb, s->st);
    launch_obs_gather<R>(d, s->obs, kind, po4, s->st);
    int npts = 0;
    HCK(hipMemcpyAsync(&npts, s->obs.n, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    launch_obs_pairs(s->obs, npts, nb, w, h.box[0], h.box[1], s->st);
    static_assert(sizeof(unsigned long long) == sizeof(int64_t), "count width");
    HCK(hipMemcpyAsync(counts, s->obs.hist, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    return MEMBX_OK;
}

int32_t membx_pair_histogram(membx_sys* s, int32_t kind, int32_t po4, const int32_t* leaflet,
                             int32_t n_bins, double bin_width, int64_t* counts)
{
    if (!s || !leaflet || !counts || n_bins < 1 || n_bins > OBS_MAXBINS || !(bin_width > 0) ||
        !std::isfinite(bin_width))
        return fail(s, MEMBX_E_INVAL, "bad arguments");
    if (kind < 0 || kind >= s->h.nk || po4 < 0 || po4 >= s->h.kn[kind])
        return fail(s, MEMBX_E_INVAL, "kind or bead index out of range");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, hist_impl, s, kind, po4, leaflet, n_bins, bin_width, counts);
    if (!rc) rc = end(s);
    return rc;
}

template <typename R>
static int32_t minimize_impl(membx_sys* s, int n_iter, double alpha, double cap)
{
    Dev<R>& d = dev<R>(s);
    for (int it = 0; it < n_iter; ++it) {
        launch_sd_step<R>(d, alpha, cap, s->st);
        refresh_forces<R>(s);
    }
    return MEMBX_OK;
}

int32_t membx_minimize(membx_sys* s, int32_t n_iter, double alpha, double max_step)
{
    if (!s || n_iter < 0 || !(alpha > 0) || !(max_step > 0))
        return fail(s, MEMBX_E_INVAL, "bad arguments");
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, minimize_impl, s, n_iter, alpha, max_step);
    if (!rc) rc = end(s);
    return rc;
}

template <typename R>
static int32_t retune_impl(membx_sys* s)
{
    Dev<R>& d = dev<R>(s);
    Host& h = s->h;
    // the grid follows the skin; counters of cells beyond the old grid are
    // cleared (the cell layout clears only the cells of the grid in use)
    set_grid(h, h.skin);
    for (int k = 0; k < 3; ++k) {
        d.nc[k] = h.nc[k]; d.ne[k] = h.ne[k];
        d.inv_edge[k] = (R)(h.nc[k] / h.box[k]);
    }
    d.ncell = h.ncell; d.next = h.next;
    HCK(hipMemsetAsync(d.cell_cnt, 0, sizeof(int) * h.ncell_cap, s->st));
    d.lpb = h.lpb;
    d.lpb_shift = h.lpb == 1 ? 0 : h.lpb == 2 ? 1 : h.lpb == 4 ? 2 : 3;
    d.bg_shift = 6 - d.lpb_shift;
    double rl = h.rc + h.skin;
    d.rl2d = rl * rl;
    set_list_band(d, h);
    d.skin_half2 = (R)(0.25 * s->h.skin * s->h.skin);
    for (auto& kv : s->gcache) (void)hipGraphExecDestroy(kv.second);
    s->gcache.clear();
    refresh_forces<R>(s);
    reset_disp<R>(s);
    HCK(hipStreamSynchronize(s->st));
    return MEMBX_OK;
}

// ---------------------------------------------------------------- autotune
// State kept across the tuning runs: slot arrays through the MDAS snapshot
// buffers, the device counters and the host mirrors.
struct Saved {
    long long ctr[NCTR];
    long long step, batch, cycle, fe, n_rebuilds;
    int since;
};

template <typename R>
static int32_t tune_save(membx_sys* s, Saved& sv)
{
    Dev<R>& d = dev<R>(s);
    launch_snapshot<R>(d, s->mv, 0, s->st);
    HCK(hipMemcpyAsync(sv.ctr, d.ctr, sizeof(sv.ctr), hipMemcpyDeviceToHost, s->st));
    HCK(hipStreamSynchronize(s->st));
    sv.step = s->step; sv.batch = s->batch; sv.cycle = s->cycle; sv.fe = s->fe;
    sv.n_rebuilds = s->n_rebuilds; sv.since = s->since;
    return MEMBX_OK;
}

template <typename R>
static int32_t tune_restore(membx_sys* s, const Saved& sv)
{
    Dev<R>& d = dev<R>(s);
    launch_fill_i32((int*)s->mv.md, 0, 16, s->st);   // restore is skipped after an accepted cycle
    launch_snapshot<R>(d, s->mv, 1, s->st);
    HCK(hipMemcpyAsync(d.ctr, sv.ctr, sizeof(sv.ctr), hipMemcpyHostToDevice, s->st));
    refresh_forces<R>(s);
    reset_disp<R>(s);
    HCK(hipStreamSynchronize(s->st));
    s->step = sv.step; s->batch = sv.batch; s->cycle = sv.cycle; s->fe = sv.fe;
    s->n_rebuilds = sv.n_rebuilds; s->since = 0;
    return MEMBX_OK;
}

// Autotuner (see membx_autotune for the search).
struct Tune {
    double skin, skin_in;
    int R, lpb, prune;
};

template <typename R>
static int32_t autotune_impl(membx_sys* s, int n, Tune* out)
{
    if (n <= 0) n = 200;
    const bool graphs0 = s->graphs;
    s->graphs = true;
    Saved sv;
    int32_t rc = tune_save<R>(s, sv);
    if (rc) return rc;
    const double skin_max = std::min(s->h.skin_max, std::floor(10.0 * box_skin_limit(s->h) + 1e-9) / 10.0);
    if (!(skin_max >= 0.1)) return fail(s, MEMBX_E_STATE, "box too small to tune the skin");
    const int lpb0 = s->h.lpb;
    auto apply = [&](const Tune& t) -> int32_t {
        s->h.skin = t.skin; s->h.R = t.R; s->h.lpb = t.lpb;
        s->h.prune = t.prune; s->h.skin_in = t.prune ? t.skin_in : 0.0;
        return retune_impl<R>(s);
    };
    // pilot: largest displacement over rebuild intervals of 4 steps
    if ((rc = apply(Tune{ skin_max, 0.0, 4, lpb0, 0 }))) return rc;
    if ((rc = md_steps<R>(s, n))) return rc;
    double d4 = 0.0;
    if ((rc = max_disp<R>(s, &d4))) return rc;
    if ((rc = tune_restore<R>(s, sv))) return rc;
    d4 = std::max(d4, 1e-6);
    hipEvent_t e0, e1;
    HCK(hipEventCreate(&e0));
    HCK(hipEventCreate(&e1));
    // candidates whose list build overflowed a lane's hit buffer come second:
    // that slower path spreads as a fresh system equilibrates and its cells
    // fill up, so their early timing flatters them
    double best_t = 1e300, best_t_ovf = 1e300;
    Tune best{ s->h.skin, s->h.skin_in, s->h.R, lpb0, s->h.prune }, best_ovf = best;
    for (int lpb : { 4, 8 }) {
        for (int sk = 2; sk <= (int)std::floor(10.0 * skin_max + 1e-9); ++sk) {
            const double skin = sk / 10.0;
            const int Rr = std::min(50, (int)std::floor(4.0 * 0.8 * 0.5 * skin / d4));
            if (Rr < 1) continue;
            for (int prune : { 0, 2, 3, 4 }) {
                Tune t{ skin, 0.0, Rr, lpb, prune };
                if (prune) {
                    if (prune >= Rr) continue;
                    // buffer keeping every bead within 0.8 delta/2 over a prune interval
                    const double din = std::ceil(100.0 * 2.0 * d4 * prune / 4.0 / 0.8) / 100.0;
                    if (din >= skin) continue;
                    t.skin_in = din;
                }
                if ((rc = apply(t))) break;
                if ((rc = md_steps<R>(s, n))) break;
                reset_disp<R>(s);
                // the fastest of three timed windows: candidates often differ
                // by a few percent, about the spread of a single window
                float ms = 1e30f;
                for (int rep = 0; rep < 3 && !rc; ++rep) {
                    HCK(hipEventRecord(e0, s->st));
                    if ((rc = md_steps<R>(s, n))) break;
                    HCK(hipEventRecord(e1, s->st));
                    HCK(hipEventSynchronize(e1));
                    float m1 = 0.f;
                    HCK(hipEventElapsedTime(&m1, e0, e1));
                    ms = std::min(ms, m1);
                }
                if (rc) break;
                double dm = 0.0;
                if ((rc = max_disp<R>(s, &dm))) break;
                int fl[NFLAGS];
                if ((rc = read_flags(s, fl))) break;
                const bool ok = fl[FL_SKIN] == 0 && fl[FL_SKIN_IN] == 0 && dm <= 0.9 * 0.5 * skin &&
                                !fl[FL_LIST_OVF] && !fl[FL_GHOST_OVF];
                if (ok && !fl[FL_HIT_OVF] && ms < best_t) { best_t = ms; best = t; }
                if (ok && fl[FL_HIT_OVF] && ms < best_t_ovf) { best_t_ovf = ms; best_ovf = t; }
                if ((rc = tune_restore<R>(s, sv))) break;
            }
            if (rc) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best_t == 1e300 && best_t_ovf < 1e300) best = best_ovf;
    if ((rc = apply(best))) return rc;
    if ((rc = tune_restore<R>(s, sv))) return rc;
    s->graphs = graphs0;
    *out = best;
    return MEMBX_OK;
}

int32_t membx_set_tuning(membx_sys* s, double skin, int32_t rebuild_interval,
                         int32_t lanes_per_bead, double skin_inner, int32_t prune_interval)
{
    if (!s) return MEMBX_E_INVAL;
    if (!(skin > 0) || skin > box_skin_limit(s->h) + 1e-12 || rebuild_interval < 1 ||
        (lanes_per_bead != 1 && lanes_per_bead != 2 && lanes_per_bead != 4 && lanes_per_bead != 8))
        return fail(s, MEMBX_E_INVAL, "bad tuning");
    const int prune = prune_interval > 1 ? prune_interval : 0;
    if (prune && (!(skin_inner > 0) || skin_inner > skin + 1e-12 || lanes_per_bead < 2))
        return fail(s, MEMBX_E_INVAL, "bad inner-list tuning");
    s->h.skin = skin;
    s->h.R = rebuild_interval;
    s->h.lpb = lanes_per_bead;
    s->h.prune = prune;
    s->h.skin_in = prune ? skin_inner : 0.0;
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, retune_impl, s);
    if (!rc) rc = end(s);
    return rc;
}

template <typename R>
static int32_t ensemble_impl(membx_sys* s)
{
    set_friction(dev<R>(s), s->h);
    HCK(hipMemcpyAsync(s->vr.kgroup, s->h.kgroup.data(), sizeof(int) * s->h.nk,
                       hipMemcpyHostToDevice, s->st));
    HCK(hipStreamSynchronize(s->st));   // the host vector may change on the next call
    for (auto& kv : s->gcache) (void)hipGraphExecDestroy(kv.second);
    s->gcache.clear();
    return MEMBX_OK;
}

template <typename R>
static int32_t regions_impl(membx_sys* s)
{
    Mv& m = s->mv;
    const Host& h = s->h;
    HCK(hipMemcpyAsync(m.region, h.region.data(), sizeof(int) * h.nm, hipMemcpyHostToDevice, s->st));
    HCK(hipMemcpyAsync(m.reg_off, h.reg_off.data(), sizeof(int) * h.reg_off.size(),
                       hipMemcpyHostToDevice, s->st));
    if (!h.reg_mem.empty())
        HCK(hipMemcpyAsync(m.reg_mem, h.reg_mem.data(), sizeof(int) * h.reg_mem.size(),
                           hipMemcpyHostToDevice, s->st));
    m.xmode = h.xmode;
    kcnt_all<R>(s);
    HCK(hipStreamSynchronize(s->st));   // the host vectors may change on the next call
    for (auto& kv : s->gcache) (void)hipGraphExecDestroy(kv.second);
    s->gcache.clear();
    return MEMBX_OK;
}

int32_t membx_set_exchange_regions(membx_sys* s, int32_t mode, const int32_t* region)
{
    if (!s) return MEMBX_E_INVAL;
    if (mode < 0 || mode > 2) return fail(s, MEMBX_E_INVAL, "exchange mode must be 0, 1 or 2");
    std::vector<int> rg(s->h.nm, 0);
    if (region)
        for (int m = 0; m < s->h.nm; ++m) {
            if (s->h.fam_of_kind[s->h.mol_kind0[m]] < 0) continue;   // never exchanged
            if (region[m] != 0 && region[m] != 1)
                return fail(s, MEMBX_E_INVAL, "regions of exchangeable molecules must be 0 or 1");
            rg[m] = region[m];
        }
    s->h.region = rg;
    s->h.xmode = mode;
    build_regions(s->h);
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, regions_impl, s);
    if (!rc) rc = end(s);
    return rc;
}

int32_t membx_set_ensemble(membx_sys* s, int32_t ensemble, double tau_t, const int32_t* kind_group)
{
    if (!s) return MEMBX_E_INVAL;
    if (ensemble != 0 && ensemble != 1) return fail(s, MEMBX_E_INVAL, "ensemble must be 0 or 1");
    if (ensemble == 1 && !(tau_t > 0.0)) return fail(s, MEMBX_E_INVAL, "tau_t must be > 0");
    std::vector<int> kg(s->h.nk, 0);
    if (kind_group)
        for (int k = 0; k < s->h.nk; ++k) {
            if (kind_group[k] != 0 && kind_group[k] != 1)
                return fail(s, MEMBX_E_INVAL, "coupling groups must be 0 or 1");
            kg[k] = kind_group[k];
        }
    s->h.ensemble = ensemble;
    s->h.tau_t = ensemble == 1 ? tau_t : 0.0;
    s->h.kgroup = kg;
    int32_t rc = begin(s);
    if (!rc) rc = DISPATCH(s, ensemble_impl, s);
    if (!rc) rc = end(s);
    return rc;
}

int32_t membx_set_barostat(membx_sys* s, int32_t nst, double p_ref_bar, double compressibility,
                           double tau_p)
{
    if (!s) return MEMBX_E_INVAL;
    if (nst > 0 && !(std::isfinite(p_ref_bar) && compressibility > 0.0 && tau_p > 0.0 &&
                     std::isfinite(compressibility) && std::isfinite(tau_p)))
        return fail(s, MEMBX_E_INVAL, "barostat needs finite p_ref, compressibility > 0, tau_p > 0");
    s->h.baro_nst = nst > 0 ? nst : 0;
    s->h.baro_kind = 0;
    s->h.p_ref = p_ref_bar / BAR;
    s->h.kappa = compressibility * BAR;
    s->h.tau_p = tau_p;
    return MEMBX_OK;
}

int32_t membx_set_barostat_pr(membx_sys* s, int32_t nst, double p_ref_bar, double compressibility,
                              double tau_p)
{
    if (!s) return MEMBX_E_INVAL;
    if (nst > 0 && !(std::isfinite(p_ref_bar) && compressibility > 0.0 && tau_p > 0.0 &&
                     std::isfinite(compressibility) && std::isfinite(tau_p)))
        return fail(s, MEMBX_E_INVAL, "barostat needs finite p_ref, compressibility > 0, tau_p > 0");
    Host& h = s->h;
    h.baro_nst = nst > 0 ? nst : 0;
    h.baro_kind = 1;
    h.p_ref = p_ref_bar / BAR;
    h.kappa = compressibility * BAR;
    h.tau_p = tau_p;
    const double lmax = std::max(h.box[0], std::max(h.box[1], h.box[2]));
    h.w_box = 3.0 * tau_p * tau_p * lmax / (4.0 * M_PI * M_PI * h.kappa);
    for (int a = 0; a < 3; ++a) h.box_v[a] = 0.0;
    return MEMBX_OK;
}

int32_t membx_barostat_state(membx_sys* s, const double* set_box_vel, double* box_vel, double* h_box)
{
    if (!s) return MEMBX_E_INVAL;
    Host& h = s->h;
    if (set_box_vel) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(set_box_vel[a])) return fail(s, MEMBX_E_NONFINITE, "non-finite box velocity");
        for (int a = 0; a < 3; ++a) h.box_v[a] = set_box_vel[a];
    }
    if (box_vel) for (int a = 0; a < 3; ++a) box_vel[a] = h.box_v[a];
    if (h_box) {
        double k = 0.0;
        for (int a = 0; a < 3; ++a) k += 0.5 * h.w_box * h.box_v[a] * h.box_v[a];
        *h_box = h.p_ref * h.box[0] * h.box[1] * h.box[2] + k;
    }
    return MEMBX_OK;
}

int32_t membx_set_mdas_path(membx_sys* s, int32_t path, double delta)
{
    if (!s) return MEMBX_E_INVAL;
    if (path != 0 && path != 1) return fail(s, MEMBX_E_INVAL, "MDAS path must be 0 or 1");
    if (path == 1 && !(delta > 0.0 && std::isfinite(delta)))
        return fail(s, MEMBX_E_INVAL, "soft-core shift must be > 0");
    s->h.mdas_path = path;
    if (path == 1) s->h.sc_delta = delta;
    return MEMBX_OK;
}

int32_t membx_get_box(membx_sys* s, double* box)
{
    if (!s || !box) return MEMBX_E_INVAL;
    for (int a = 0; a < 3; ++a) box[a] = s->h.box[a];
    return MEMBX_OK;
}

int32_t membx_set_graphs(membx_sys* s, int32_t enable)
{
    if (!s) return MEMBX_E_INVAL;
    s->graphs = enable != 0;
    return MEMBX_OK;
}

int32_t membx_kernel_timing(membx_sys* s, int32_t enable)
{
    if (!s) return MEMBX_E_INVAL;
    s->timing = enable != 0;
    s->tev_used = 0;
    s->t_launches = 0;
    s->t_ms = 0.0;
    return MEMBX_OK;
}

int32_t membx_kernel_time(membx_sys* s, int64_t* launches, double* mean_ms)
{
    if (!s) return MEMBX_E_INVAL;
    HCK(hipStreamSynchronize(s->st));
    for (size_t q = 0; q < s->tev_used; ++q) {
        float ms = 0.f;
        HCK(hipEventElapsedTime(&ms, s->tev[q].first, s->tev[q].second));
        s->t_ms += ms;
        s->t_launches++;
    }
    s->tev_used = 0;
    if (launches) *launches = s->t_launches;
    if (mean_ms) *mean_ms = s->t_launches ? s->t_ms / s->t_launches : 0.0;
    return MEMBX_OK;
}

template <typename R>
static int32_t kbench_impl(membx_sys* s, int n, double* mean_ms)
{
    Dev<R>& d = dev<R>(s);
    hipGraph_t g;
    if (hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(s, MEMBX_E_DEVICE, "stream capture failed");
    // the kernel most MD steps run: forces plus the next step's update (the
    // inner-list walk when pruning is on), the update written to scratch
    // (the other coordinate buffer, the sort buffer for velocities) so that
    // the state is unchanged; right after a rebuild the inner list is stale,
    // which changes the values, not the work
    const int list = (s->h.prune > 1 && s->h.lpb >= 2) ? 1 : 0;
    for (int q = 0; q < n; ++q)
        launch_nonbonded_fused<R>(d, s->h.lpb, list, (R)s->h.dt, 1, d.posq_alt, d.vel_t, 0, s->st);
    if (hipStreamEndCapture(s->st, &g) != hipSuccess)
        return fail(s, MEMBX_E_DEVICE, "stream capture failed");
    hipGraphExec_t ge;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(s, MEMBX_E_DEVICE, "graph instantiation failed");
    }
    (void)hipGraphDestroy(g);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    hipError_t e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s->st);
    if (e == hipSuccess) e = hipEventRecord(e0, s->st);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s->st);
    if (e == hipSuccess) e = hipEventRecord(e1, s->st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGraphExecDestroy(ge);
    if (e != hipSuccess) return fail(s, MEMBX_E_DEVICE, hipGetErrorString(e));
    *mean_ms = (double)ms / n;
    return MEMBX_OK;
}

int32_t membx_kernel_bench(membx_sys* s, int32_t n_launch, double* mean_ms)
{
    if (!s || !mean_ms || n_launch < 1 || n_launch > 4096) return fail(s, MEMBX_E_INVAL, "bad arguments");
    int32_t rc = begin(s);
    if (rc) return rc;
    rc = DISPATCH(s, kbench_impl, s, n_launch, mean_ms);
    if (!rc) rc = end(s);
    return rc;
}

const char* membx_last_error(const membx_sys* s) { return s ? s->err.c_str() : ""; }

int32_t membx_status(membx_sys* s)
{
    if (!s) return MEMBX_E_INVAL;
    int fl[NFLAGS];
    int32_t rc = read_flags(s, fl);
    if (rc) return rc;
    return flag_status(s, fl);
}

int32_t membx_calib_copy(membx_sys* s, void* dst, const void* src, uint64_t bytes)
{
    if (!s || !dst || !src || bytes % 16) return fail(s, MEMBX_E_INVAL, "bad arguments");
    int32_t rc = begin(s);
    if (rc) return rc;
    launch_copy(dst, src, bytes, s->st);
    return end(s);
}

int32_t membx_autotune(membx_sys* s, int32_t n_steps, double* skin, int32_t* rebuild_interval,
                       int32_t* lanes_per_bead, double* skin_inner, int32_t* prune_interval)
{
    if (!s) return MEMBX_E_INVAL;
    int32_t rc = begin(s);
    if (rc) return rc;
    Tune t{};
    const int nst0 = s->h.baro_nst;   // the timing runs keep the box
    s->h.baro_nst = 0;
    rc = DISPATCH(s, autotune_impl, s, n_steps, &t);
    s->h.baro_nst = nst0;
    if (!rc) rc = end(s);
    if (rc) return rc;
    if (skin) *skin = t.skin;
    if (rebuild_interval) *rebuild_interval = t.R;
    if (lanes_per_bead) *lanes_per_bead = t.lpb;
    if (skin_inner) *skin_inner = t.skin_in;
    if (prune_interval) *prune_interval = t.prune;
    return MEMBX_OK;
}


// ================================================================== serving
// Jobs resident in one caller-owned arena, each on its own stream.  The
// arena is managed by a first-fit free list (offset -> size, coalesced on
// release); admission is strictly first come, first served.

namespace {

constexpr int SRV_DEPTH = 2;   // cycles in flight per job

struct SrvJob {
    int64_t id = 0;
    membx_sys* s = nullptr;       // host part prepared at submit
    membx_request rq{};
    std::vector<double> pos, vel;
    uint64_t bytes = 0;
    size_t off = 0, span = 0;     // arena block
    bool resident = false;
    double t_submit = 0, t_admit = 0;
    int total = 0, issued = 0, done = 0;
    int32_t status = MEMBX_OK;
    hipEvent_t ev[SRV_DEPTH][2] = {};
    std::deque<int> inflight;     // event slots of cycles in flight
    int next_slot = 0;
    std::vector<float> cyc;
    // pair counting (request.count_pairs): energy-pass sums of each slot's
    // cycle land in pinned host memory, read when the cycle's event is done
    double* sums = nullptr;       // SRV_DEPTH x 16 doubles
    int64_t slot_steps[SRV_DEPTH] = {};
    int64_t pair_int = 0;
};

// Energy pass at the end of a cycle: its sums (in-cutoff pair count at
// index 5) are copied to host slot memory on the job's stream.
template <typename R>
static void srv_count_pairs(membx_sys* s, double* host)
{
    Dev<R>& d = dev<R>(s);
    const int nnb = launch_nonbonded<R>(d, s->h.lpb, true, d.red, s->st);
    launch_energy_final(d.red, nnb, d.eout, s->st);
    (void)hipMemcpyAsync(host, d.eout, sizeof(double) * 13, hipMemcpyDeviceToHost, s->st);
}

}  // namespace

struct membx_server {
    char* base = nullptr;
    uint64_t bytes = 0;
    std::map<size_t, size_t> free_;        // offset -> size
    std::deque<SrvJob*> queue;
    std::vector<SrvJob*> active;
    std::deque<membx_job_result> finished;
    std::vector<float> cycles;
    std::vector<double> cycle_pairs;       // pair interactions of each cycle (-1: not counted)
    int64_t next_id = 1;
    std::chrono::steady_clock::time_point t0;
    std::string err;
    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static bool srv_alloc(membx_server* v, size_t n, size_t* off)
{
    for (auto it = v->free_.begin(); it != v->free_.end(); ++it) {
        if (it->second >= n) {
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t at = it->first + n;
            v->free_.erase(it);
            if (rest) v->free_[at] = rest;
            return true;
        }
    }
    return false;
}

static void srv_release(membx_server* v, size_t off, size_t n)
{
    auto it = v->free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != v->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        v->free_.erase(nx);
    }
    if (it != v->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            v->free_.erase(it);
        }
    }
}

static double pct(std::vector<float> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = (size_t)std::ceil(q * (double)v.size()) - 1;
    if (k >= v.size()) k = v.size() - 1;
    return v[k];
}

int32_t membx_server_create(void* dev_arena, uint64_t arena_bytes, membx_server** out)
{
    if (!out || !dev_arena || arena_bytes < 4096) return MEMBX_E_INVAL;
    membx_server* v = new membx_server();
    // 256-byte aligned usable range
    const uintptr_t b = ((uintptr_t)dev_arena + 255) / 256 * 256;
    v->base = (char*)b;
    v->bytes = arena_bytes - (b - (uintptr_t)dev_arena);
    v->bytes = v->bytes / 256 * 256;
    v->free_[0] = v->bytes;
    v->t0 = std::chrono::steady_clock::now();
    *out = v;
    return MEMBX_OK;
}

int32_t membx_server_submit(membx_server* v, const membx_desc* desc, const membx_request* rq,
                            int64_t* job_id)
{
    if (!v || !desc || !rq) return MEMBX_E_INVAL;
    if (rq->minimize_iters < 0 || rq->md_cycles < 0 || rq->mdas_cycles < 0 ||
        rq->md_cycles + rq->mdas_cycles <= 0 ||
        (rq->md_cycles > 0 && rq->md_steps < 1) ||
        (rq->mdas_cycles > 0 && (rq->mdas_pairs < 1 || rq->mdas_k < 1 || rq->mdas_m < 0)) ||
        (rq->count_pairs != 0 && rq->count_pairs != 1)) {
        v->err = "bad request";
        return MEMBX_E_INVAL;
    }
    SrvJob* j = new SrvJob();
    j->s = new membx_sys();
    Status st = check_desc(desc, j->s->h);
    if (!st.code) st = derive(desc, j->s->h);
    if (!st.code && rq->mdas_cycles > 0 && (rq->mdas_pairs > j->s->h.P_cap || j->s->h.sw_list.empty()))
        st = { MEMBX_E_INVAL, "MDAS request not possible for this system" };
    if (st.code) {
        v->err = st.msg;
        delete j->s;
        delete j;
        return st.code;
    }
    membx_sys* s = j->s;
    j->bytes = s->mixed() ? layout<float>(s, s->df, s->mv, nullptr) : layout<double>(s, s->dd, s->mv, nullptr);
    j->span = (j->bytes + 255) / 256 * 256;
    if (j->span > v->bytes) {
        v->err = "job larger than the server arena";
        delete j->s;
        delete j;
        return MEMBX_E_NOMEM;
    }
    const size_t n3 = 3 * (size_t)s->h.N;
    j->pos.assign(desc->pos, desc->pos + n3);
    if (desc->vel) j->vel.assign(desc->vel, desc->vel + n3);
    j->rq = *rq;
    j->total = rq->md_cycles + rq->mdas_cycles;
    j->id = v->next_id++;
    j->t_submit = v->now();
    v->queue.push_back(j);
    if (job_id) *job_id = j->id;
    return MEMBX_OK;
}

// Build the job's device state in its block (on its own stream).
static int32_t srv_admit(membx_server* v, SrvJob* j)
{
    membx_sys* s = j->s;
    char* base = v->base + j->off;
    if (s->mixed()) layout<float>(s, s->df, s->mv, base);
    else layout<double>(s, s->dd, s->mv, base);
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming) != hipSuccess)
        return MEMBX_E_DEVICE;
    s->user = s->st;   // a job is ordered only against itself
    for (int q = 0; q < SRV_DEPTH; ++q)
        if (hipEventCreateWithFlags(&j->ev[q][0], hipEventDisableSystemFence) != hipSuccess ||
            hipEventCreate(&j->ev[q][1]) != hipSuccess)
            return MEMBX_E_DEVICE;
    if (j->rq.count_pairs &&
        hipHostMalloc((void**)&j->sums, sizeof(double) * 16 * SRV_DEPTH, hipHostMallocDefault) != hipSuccess)
        return MEMBX_E_DEVICE;
    membx_desc dsc{};
    dsc.pos = j->pos.data();
    dsc.vel = j->vel.empty() ? nullptr : j->vel.data();
    int32_t rc = DISPATCH(s, upload, s, &dsc);
    if (!rc && j->rq.minimize_iters > 0) rc = membx_minimize(s, j->rq.minimize_iters, 1e-4, 0.01);
    return rc;
}

static int32_t srv_issue(SrvJob* j)
{
    membx_sys* s = j->s;
    const int slot = j->next_slot;
    j->next_slot = (j->next_slot + 1) % SRV_DEPTH;
    if (hipEventRecord(j->ev[slot][0], s->st) != hipSuccess) return MEMBX_E_DEVICE;
    int32_t rc;
    if (j->issued < j->rq.md_cycles) {
        rc = membx_md_step(s, j->rq.md_steps);
        j->slot_steps[slot] = j->rq.md_steps;
    } else {
        rc = membx_mdas_cycle(s, j->rq.mdas_pairs, j->rq.mdas_k, j->rq.mdas_m, nullptr, nullptr, nullptr);
        j->slot_steps[slot] = (int64_t)j->rq.mdas_k * j->rq.mdas_m;
    }
    if (rc) return rc;
    if (j->sums) {
        if (s->mixed()) srv_count_pairs<float>(s, j->sums + 16 * slot);
        else srv_count_pairs<double>(s, j->sums + 16 * slot);
    }
    if (hipEventRecord(j->ev[slot][1], s->st) != hipSuccess) return MEMBX_E_DEVICE;
    j->inflight.push_back(slot);
    j->issued++;
    return MEMBX_OK;
}

static void srv_free_job(membx_server* v, SrvJob* j)
{
    if (j->resident) {
        if (j->s->st) (void)hipStreamSynchronize(j->s->st);
        for (int q = 0; q < SRV_DEPTH; ++q)
            for (int e = 0; e < 2; ++e)
                if (j->ev[q][e]) (void)hipEventDestroy(j->ev[q][e]);
        srv_release(v, j->off, j->span);
    }
    if (j->sums) (void)hipHostFree(j->sums);
    membx_sys_destroy(j->s);
    delete j;
}

static void srv_close(membx_server* v, SrvJob* j)
{
    membx_job_result r{};
    r.job_id = j->id;
    r.status = j->status;
    r.n_cycles = j->done;
    r.n_beads = j->s->h.N;
    r.submit_s = j->t_submit;
    r.admit_s = j->t_admit;
    r.cycle_ms_p50 = pct(j->cyc, 0.50);
    r.cycle_ms_p99 = pct(j->cyc, 0.99);
    r.cycle_ms_max = pct(j->cyc, 1.0);
    r.pair_interactions = j->sums ? j->pair_int : -1;
    if (j->status == MEMBX_OK) {
        membx_energy e{};
        int32_t rc = membx_energies(j->s, &e);
        long long ctr[NCTR] = { 0, 0, 0, 0 };
        const long long* dctr = j->s->mixed() ? j->s->df.ctr : j->s->dd.ctr;
        if (hipMemcpy(ctr, dctr, sizeof(ctr), hipMemcpyDeviceToHost) != hipSuccess) rc = MEMBX_E_DEVICE;
        r.status = rc;
        r.potential = e.potential;
        r.pairs_in_cutoff = e.n_pairs_in_cutoff;
        r.fe_count = e.fe_count;
        r.md_steps = ctr[CT_STEP];
        r.mdas_accepted = (int32_t)ctr[CT_MDAS_ACC];
    }
    r.finish_s = v->now();
    v->finished.push_back(r);
    srv_free_job(v, j);
}

int32_t membx_server_poll(membx_server* v, membx_job_result* out, int32_t cap, int32_t* n_out,
                          int32_t* n_resident, int32_t* n_waiting)
{
    if (!v || cap < 0 || (cap > 0 && !out)) return MEMBX_E_INVAL;
    // 1. collect finished cycles; close finished jobs
    for (size_t q = 0; q < v->active.size();) {
        SrvJob* j = v->active[q];
        while (!j->inflight.empty()) {
            const int slot = j->inflight.front();
            const hipError_t e = hipEventQuery(j->ev[slot][1]);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) { j->status = MEMBX_E_DEVICE; j->inflight.clear(); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, j->ev[slot][0], j->ev[slot][1]);
            j->cyc.push_back(ms);
            v->cycles.push_back(ms);
            if (j->sums) {
                const int64_t pairs = (int64_t)std::llround(j->sums[16 * slot + 5]);
                j->pair_int += pairs * j->slot_steps[slot];
                v->cycle_pairs.push_back((double)pairs * (double)j->slot_steps[slot]);
            } else {
                v->cycle_pairs.push_back(-1.0);
            }
            j->inflight.pop_front();
            j->done++;
        }
        const bool over = j->inflight.empty() && (j->done >= j->total || j->status != MEMBX_OK);
        if (over) {
            v->active.erase(v->active.begin() + q);
            srv_close(v, j);
        } else {
            ++q;
        }
    }
    // 2. admit waiting jobs in order while their blocks fit
    while (!v->queue.empty()) {
        SrvJob* j = v->queue.front();
        size_t off = 0;
        if (!srv_alloc(v, j->span, &off)) break;
        v->queue.pop_front();
        j->off = off;
        j->resident = true;
        j->t_admit = v->now();
        const int32_t rc = srv_admit(v, j);
        if (rc) {
            j->status = rc;
            v->err = "admission failed: " + j->s->err;
            srv_close(v, j);
            continue;
        }
        v->active.push_back(j);
    }
    // 3. keep up to SRV_DEPTH cycles in flight per job
    for (SrvJob* j : v->active)
        while (j->status == MEMBX_OK && j->issued < j->total && (int)j->inflight.size() < SRV_DEPTH) {
            const int32_t rc = srv_issue(j);
            if (rc) { j->status = rc; v->err = j->s->err; }
        }
    int32_t n = 0;
    while (n < cap && !v->finished.empty()) {
        out[n++] = v->finished.front();
        v->finished.pop_front();
    }
    if (n_out) *n_out = n;
    if (n_resident) *n_resident = (int32_t)v->active.size();
    if (n_waiting) *n_waiting = (int32_t)v->queue.size();
    return MEMBX_OK;
}

int32_t membx_server_cycle_times(membx_server* v, float* out, int64_t cap, int64_t* n)
{
    if (!v || cap < 0 || (cap > 0 && !out)) return MEMBX_E_INVAL;
    const int64_t m = std::min<int64_t>(cap, (int64_t)v->cycles.size());
    for (int64_t q = 0; q < m; ++q) out[q] = v->cycles[q];
    if (n) *n = (int64_t)v->cycles.size();
    return MEMBX_OK;
}

int32_t membx_server_cycle_pairs(membx_server* v, double* out, int64_t cap, int64_t* n)
{
    if (!v || cap < 0 || (cap > 0 && !out)) return MEMBX_E_INVAL;
    const int64_t m = std::min<int64_t>(cap, (int64_t)v->cycle_pairs.size());
    for (int64_t q = 0; q < m; ++q) out[q] = v->cycle_pairs[q];
    if (n) *n = (int64_t)v->cycle_pairs.size();
    return MEMBX_OK;
}

int32_t membx_server_destroy(membx_server* v)
{
    if (!v) return MEMBX_OK;
    for (SrvJob* j : v->active) srv_free_job(v, j);
    for (SrvJob* j : v->queue) srv_free_job(v, j);
    delete v;
    return MEMBX_OK;
}

const char* membx_server_last_error(const membx_server* v) { return v ? v->err.c_str() : ""; }
