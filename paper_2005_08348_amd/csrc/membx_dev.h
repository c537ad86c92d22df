// membx_dev.h -- device-side types and helpers of the membx library
// (gfx950 / CDNA4, wave64).  Shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbx {

constexpr int WG = 256;          // work-group size of the per-bead kernels
constexpr int MAXEXCL = 8;       // bonded partners per bead (nrexcl = 1)
constexpr int MAXCLS = 16;       // distinct (bead type, charge) classes
constexpr int MAXCH = 8;         // beads changed per molecule by an exchange
constexpr int MAXMB = 16;        // beads per bonded molecule
constexpr int CODE_SHIFT = 29;   // neighbour entry: j | (i-shift bits << 29)
constexpr int JMASK = (1 << CODE_SHIFT) - 1;
constexpr int MAXBT = 8;         // bonded terms per bead

// random streams (fourth Philox counter word)
enum { ST_LANGEVIN = 0, ST_SWAP_DRAW = 1, ST_SWAP_ACCEPT = 2, ST_MDAS_SELECT = 3,
       ST_MDAS_ACCEPT = 4, ST_VRESCALE = 5, ST_BARO = 6 };

// device flags
// FL_SKIN counts (bead, step) events beyond skin/2 since the last reset;
// FL_SKIN_IN the same for the inner list (beyond delta/2 since its prune);
// FL_HIT_OVF: a list-build lane overflowed its hit buffer and took the
// slower re-test path since the last reset (not an error);
// FL_LIST_NEED: the largest entry count a bead needed when FL_LIST_OVF was
// raised (the capacity that would have held its list)
enum { FL_LIST_OVF = 0, FL_SKIN = 1, FL_GHOST_OVF = 2, FL_NONFINITE = 3, FL_AFF_OVF = 4,
       FL_REBUILDS = 5, FL_SKIN_IN = 6, FL_HIT_OVF = 7, FL_LIST_NEED = 8, NFLAGS = 9 };

// The 8 XCDs of the chip take work-groups round-robin by id, each with its
// own L2, and an XCD deals its work-groups round-robin to its 32 CUs.
// xcd_block(b, n) renumbers work-group b of n so that every XCD runs one
// contiguous range of logical blocks (a slab of neighbouring cells), whose
// coordinate gathers stay in its own L2, and within it every CU a
// contiguous sub-range, so that the work-groups resident on a CU share
// neighbourhoods in its L1 (measured on the 95,876-bead bilayer: force pass
// 20.2 -> 19.9 us at skin 0.3 nm, 23.0 -> 21.9 us at 0.4 nm).  A bijection
// of [0, n).
constexpr int NXCD = 8;
constexpr int CU_PER_XCD = 32;
__device__ __forceinline__ int split_rr(int b, int n, int k)
{
    // work-group b of n dealt round-robin to k units; unit b % k runs the
    // (b / k)-th block of its own contiguous range
    const int x = b % k, l = b / k, per = n / k, rem = n % k;
    return x < rem ? x * (per + 1) + l : rem * (per + 1) + (x - rem) * per + l;
}
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int x = b % NXCD, per = n / NXCD, rem = n % NXCD;
    const int nx = x < rem ? per + 1 : per;
    const int base = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return base + split_rr(b / NXCD, nx, CU_PER_XCD);
}

// device counters (int64)
enum { CT_STEP = 0, CT_BATCH = 1, CT_CYCLE = 2, CT_MDAS_ACC = 3, NCTR = 4 };

template <typename R> struct alignas(4 * sizeof(R)) V4 { R x, y, z, w; };

template <typename R> __device__ __forceinline__ int cls_of(R w);
template <> __device__ __forceinline__ int cls_of<float>(float w) { return __float_as_int(w); }
template <> __device__ __forceinline__ int cls_of<double>(double w)
{
    return (int)__double2loint(w);
}
template <typename R> __device__ __forceinline__ R cls_to(int c);
template <> __device__ __forceinline__ float cls_to<float>(int c) { return __int_as_float(c); }
template <> __device__ __forceinline__ double cls_to<double>(int c)
{
    return __hiloint2double(0, c);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products of counter words 0 and 2 with the published
// multipliers, mixing in the other words and the key; the key advances by
// the Weyl increments between rounds.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t index, int64_t ctr, uint32_t stream)
{
    return philox(index, (uint32_t)((uint64_t)ctr), (uint32_t)((uint64_t)ctr >> 32), stream,
                  (uint32_t)seed, (uint32_t)(seed >> 32));
}

// uniform in [0,1) with 53 bits: ((a >> 5) 2^26 + (b >> 6)) 2^-53
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ uint32_t pick(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

// Box-Muller: three normals from one block; u1 = (w+1)/2^32 in (0,1].
template <typename R> __device__ __forceinline__ void gauss3(uint4 w, R g[3]);
template <> __device__ __forceinline__ void gauss3<double>(uint4 w, double g[3])
{
    const double s32 = 1.0 / 4294967296.0, tp = 6.283185307179586476925286766559;
    double r1 = sqrt(-2.0 * log(((double)w.x + 1.0) * s32));
    double r2 = sqrt(-2.0 * log(((double)w.z + 1.0) * s32));
    double sn, cs;
    sincos(tp * ((double)w.y * s32), &sn, &cs);
    g[0] = r1 * cs;
    g[1] = r1 * sn;
    g[2] = r2 * cos(tp * ((double)w.w * s32));
}
// float32 form: the top 24 bits of each word ((w >> 8) + 1) 2^-24 in (0,1]
template <> __device__ __forceinline__ void gauss3<float>(uint4 w, float g[3])
{
    const float s24 = 1.0f / 16777216.0f, tp = 6.2831853071795864769f;
    float r1 = sqrtf(-2.0f * logf((float)((w.x >> 8) + 1u) * s24));
    float r2 = sqrtf(-2.0f * logf((float)((w.z >> 8) + 1u) * s24));
    float sn, cs;
    sincosf(tp * ((float)(w.y >> 8) * s24), &sn, &cs);
    g[0] = r1 * cs;
    g[1] = r1 * sn;
    g[2] = r2 * cosf(tp * ((float)(w.w >> 8) * s24));
}

// Pair-parameter tables, indexed [ci * MAXCLS + cj]:
//   force  : {6 C6, 12 C12, f qi qj / eps_r, 2 k_rf f qi qj / eps_r}
//   energy : {C6, C12, f qi qj / eps_r, C12/rc^12 - C6/rc^6}
// so that  F/r = (12 C12 r^-12 - 6 C6 r^-6) r^-2 + qq (r^-3 - 2 k_rf)
//          V   = C12 r^-12 - C6 r^-6 - shift + qq (1/r + k_rf r^2 - c_rf).

// Buffers of the mixing observable (pair histogram of PO4 beads).
constexpr int OBS_MAXBINS = 4096;
struct ObsBuf {
    int* leaf;                 // [nm] leaflet of each molecule (-1: skip), from the caller
    double2* xy;               // [nm] selected PO4 coordinates (x, y)
    int* lf;                   // [nm] their leaflets
    int* n;                    // [1] selected count
    double* edge2;             // [OBS_MAXBINS + 1] squared bin edges
    unsigned long long* hist;  // [OBS_MAXBINS] pair counts
};

// Boundary between two MDAS segments fused into the force pass (linear
// path, Langevin): the affected beads' force difference F_B - F_A (dfrc,
// computed beforehand at the same coordinates) and the two lambdas' weights.
template <typename R> struct AlchK {
    const int* aff_flag;   // [N] nonzero: the bead's force depends on lambda
    double* md;            // MDAS accumulators: md[0] += dlw md[1] (work)
    R lam, dl;             // lambda of the closing step, increment to the next
    double dlw;
};

// Stochastic velocity rescaling with two coupling groups: the group of a
// bead is kgroup[kind of its molecule], so it follows exchanges of kinds.
struct VrBuf {
    int* bmol;       // [N] molecule of each bead (bead-id order)
    int* kgroup;     // [nk] coupling group (0/1) of each molecule kind
    double* part;    // [4 * blocks] per block: K of group 0, 1; beads of group 0, 1
    double* alpha;   // [2] velocity factors of the step
};

// Everything a kernel needs about one system (passed by value).
template <typename R> struct Dev {
    // sizes
    int N, Npad, nm, nk, ncls, Kcap, Gcap, nbm;
    // box and cutoffs
    R L[3], halfL[3];
    double Ld[3];
    R rc2, krf, crf;
    double rc2d, rl2d;
    R rl2_lo, rl2_hi;     // list prefilter band around (r_cut + skin)^2
    R skin_half2;
    // dynamics
    R dt, half_dt, c1, c2, kT;
    double kTd;
    uint64_t seed;
    // cell grid (real cells nc, extended grid ne = nc + 1 with a halo layer at 0)
    int nc[3], ncell, ne[3], next;
    R inv_edge[3];
    // per-slot state (sorted order)
    V4<R>* posq;     // [N + Gcap], w = class bits (current coordinates)
    V4<R>* posq_alt; // [N + Gcap] the other coordinate buffer: the force kernel
                     // that also integrates reads posq and writes the new
                     // coordinates here, then the two are exchanged
    V4<R>* vel;      // [N], w = 1/m
    V4<R>* frc;      // [N]
    V4<R>* xref;     // [N] positions at the last rebuild
    V4<R>* dfrc;     // [N] alchemical force difference F_B - F_A (sparse use)
    int* orig;       // slot -> bead id
    int* inv;        // bead id -> slot
    int* alch;       // slot -> -1 or (new class | trial << 8)
    // sort scratch
    V4<R>* posq_t;
    V4<R>* vel_t;
    V4<R>* frc_t;
    int* orig_t;
    int* alch_t;
    int* cell_t;     // [N] cell of each slot (binning)
    int* cell_pos;   // [N] its place in the cell (binning, arbitrary order)
    int* cell_cnt;   // [ncell]
    int* cell_start; // [ncell + 1]
    int* ext_start;  // [next]
    int* ext_cnt;    // [next]
    int* ext_scan;   // [next + 1]
    int* ghost_owner;  // [Gcap] slot whose image each ghost is
    int* n_ghost;    // [1]
    int* glist;      // [N * 8] their ghost indices | code << 29, -1 unused
    int* orig_ext;   // [N + Gcap] bead id of each slot or ghost image
    int4* bslot;     // [N * 8] bonded terms of each slot with partner slots
                     // {role, slot 1, slot 2, parameter}; role -1 = unused
    float* dmax_part;  // [ceil(8 N / WG)] per integrator block: largest squared
                       // displacement from the last rebuild seen since a reset
    // neighbour list, tiled so that the LPB lanes of the 64/LPB beads a wave
    // handles read one contiguous 256-byte block per load (see nbr_index)
    int lpb, lpb_shift, bg_shift;   // lanes per bead, log2(lpb), log2(64/lpb)
    int* nbr;
    int* ncnt;
    // inner (pruned) list, same layout and capacity: the entries of the
    // outer list within r_cut + delta at the last prune (coordinates xref_in)
    int* nbr_in;
    int* ncnt_in;
    V4<R>* xref_in;
    R rin2;          // (r_cut + delta)^2; 0: no inner list
    R in_half2;      // (delta / 2)^2
    int* nseg0;
    // topology
    int* excl;       // [N * MAXEXCL] bead ids, -1 padded
    unsigned* exmask;  // [N] bit (j - i + 16) set when bead j is bonded to bead i
    int* mol_first;  // [nm]
    int* mol_kind;   // [nm] current kinds
    int* bmols;      // [nbm] molecules with bonded terms
    int* kn;         // [nk]
    int* kbead_off;  // [nk]
    int* kcls;       // [sum kn] class of each kind bead
    int* kb_off; int* kb_n; int* b_ij; R* b_par;   // bonds: (i,j), (b0,k)
    int* ka_off; int* ka_n; int* a_ijk; R* a_par;  // angles: (i,j,k), (cos0,k)
    // bonded terms seen from each bead (bead-id order): [bt_off[b], bt_off[b+1])
    // entries {role, partner 1, partner 2, parameter index}; roles: 0 bond
    // (energy owner), 1 bond, 2 angle end, 3 angle vertex (energy owner)
    int* bt_off;
    int4* bt;
    R* bt_par;       // (b0, k) or (cos theta0, k)
    // topology-changing exchanges (kinds of one family with different
    // bonded terms): topo != 0; ktopo[k1 * nk + k2] marks such kind pairs;
    // the bonded terms then sit MAXBT per bead (bt_off[b] = b MAXBT) and are
    // rewritten from the per-kind templates ktpl[(kbead_off[k] + l) MAXBT
    // + t] = {role, partner 1, partner 2 (-1: none), parameter} in local
    // bead indices when a molecule changes kind
    int topo;
    int* ktopo;
    int4* ktpl;
    // tables
    V4<R>* tabF;
    V4<R>* tabE;
    // flags / counters / reductions
    int* flags;
    long long* ctr;
    double* red;     // block partials
    double* eout;    // final energies
};

// coupling group (0/1) of the bead in slot i under velocity rescaling
template <typename R>
__device__ __forceinline__ int vr_group(const Dev<R>& d, const VrBuf& vr, int i)
{
    return vr.kgroup[d.mol_kind[vr.bmol[d.orig[i]]]];
}

// Exchange moves (batched MC-MD trials and MDAS pair selection) and the
// sparse alchemical force / energy difference machinery.
constexpr int SEL_C0 = 1024;     // candidates of the first selection chunk
constexpr int SEL_CMAX = 8192;   // largest selection chunk
constexpr int SEL_CAPC = 64;     // earlier conflicting candidates listed per candidate
constexpr int SEL_LDS = 61440;   // conflict-list entries one chunk may resolve (120 KB of LDS)
constexpr int MAXMC = 2 * MAXCH; // changed beads per trial
constexpr int MAXKN_TOPO = 16;   // beads per molecule in a topology-changing family
// selection state words
enum { SEL_ADM = 0, SEL_NEXT = 1, SEL_DONE = 2, SEL_EPC = 3, SEL_STAMP = 4, SEL_NSEL = 8 };
constexpr int HBW = 4;           // entries per hash bucket
struct Mv {
    // static tables
    int n_sw;            // exchangeable molecules
    int* sw_list;        // [n_sw] ascending molecule ids
    int* fam_of_kind;    // [nk] (-1: none)
    int* fam_off;        // [nfam + 1] offsets into fam_mem
    int* fam_mem;        // family members, ascending molecule ids
    int fam_stride;      // max family size + 1
    int* kcnt;           // [nk * fam_stride] per-kind prefix counts over its family
    int* others;         // [nk * fam_stride] family members of another kind, ascending
    // exchange regions (leaflets): xmode 0 partners anywhere in the family,
    // 1 of another kind within X's region, 2 any member in the other region
    int xmode;
    int* region;         // [nm] 0/1
    int* reg_off;        // [2 nfam + 1] offsets of (family, region) into reg_mem
    int* reg_mem;        // family members by region, ascending molecule ids
    int* kcnt_r;         // [nk * 2 * fam_stride] kcnt over the members of one region
    int* others_r;       // [nk * 2 * fam_stride] others within one region
    int* chg_n;          // [nk * nk] changed beads between two kinds
    int* chg_loc;        // [nk * nk * MAXCH] their local indices
    int maxcht;          // max changed beads per trial (both molecules)
    // candidate scratch (one chunk of up to SEL_CMAX draws)
    int* c_x; int* c_y; int* c_nb; int* c_flag;               // [SEL_CMAX]
    int* c_bead; int* c_cls;                                  // [SEL_CMAX * maxcht]
    double* c_pos;       // [SEL_CMAX * maxcht * 3]
    int* c_conf_n; int* c_conf;                               // [SEL_CMAX], [SEL_CMAX * SEL_CAPC]
    // spatial hashes over the box (cells of edge >= r_cut): open addressing,
    // one 64-bit word per bucket {epoch:32, key:24, count:8} and up to HBW
    // entries; a key with more entries continues in the following buckets.
    // hb: changed beads of the chunk's live candidates (entry = t*maxcht+q);
    // ab: changed beads of the trials admitted so far (entry = a*maxcht+q);
    // mb: molecules of the chunk's live candidates (entry = 2t or 2t+1)
    int hnc[3], hcells;
    double hinv[3];
    unsigned long long* hb_word; int* hb_ent; int hb_mask;
    unsigned long long* ab_word; int* ab_ent; int ab_mask;
    unsigned long long* mb_word; int* mb_ent; int mb_mask;
    int* used;           // [nm] stamp of the call that admitted the molecule
    int* sel;            // [SEL_NSEL] selection state
    // results (capacity T = max(max_trials, max_pairs))
    int T;
    int* r_n;            // [4]: admitted, draws, -, accepted
    int* r_draw; int* r_x; int* r_y; int* r_acc;
    double* r_du; double* r_u;
    int* r_nb; int* r_bead; int* r_cls;                       // changed beads per trial
    double* r_pos;       // [T * maxcht * 3] their positions at selection
    double* du_bead;     // [T * maxcht]
    // affected set
    int* aff_flag;       // [N]
    int* aff_list;       // [aff_cap]
    int* aff_n;          // [1]
    int aff_cap;
    // bonded part of an exchange that changes the topology: dU per trial
    // (scaled as the caller asks; zero otherwise) and F_B - F_A on the
    // beads of each exchanged molecule ([T][2][MAXKN_TOPO][3])
    double* du_bond;     // [T]
    double* dfb;
    // MDAS
    double* md;          // [8]: work, dU, accept, u
    double* dsc;         // [4 N] soft-core force change of an affected bead between
                         // two lambdas, held for the segment boundary pass
    // snapshot of the per-slot state
    void* snap_posq; void* snap_vel; void* snap_frc; int* snap_orig;
};

// One bead through B (kick, folding in the closing B of the previous step) +
// A + O (Ornstein-Uhlenbeck with Philox noise) + A of a BAOAB step; the new
// coordinates go to pos_out (the bead's slot and its periodic images, which
// are exact shifts by -L), the velocity to vel_out.  Returns the squared
// displacement from the coordinates of the last list build, and (chk_in:
// the inner list is valid) in e2_in the one from its last prune.
// Per-bead inputs of baoab_bead that do not depend on the force, loaded
// early by the force kernel so that they are in flight with its first reads.
template <typename R> struct BeadPre {
    V4<R> v, xr, xri;
    int orig;
    int4 g0;
};

template <typename R>
__device__ __forceinline__ BeadPre<R> bead_pre(const Dev<R>& d, int i, bool chk_in)
{
    BeadPre<R> b;
    b.v = d.vel[i];
    b.xr = d.xref[i];
    b.xri = chk_in ? d.xref_in[i] : b.xr;
    b.orig = d.orig[i];
    b.g0 = reinterpret_cast<const int4*>(d.glist)[2 * i];
    return b;
}

template <typename R>
__device__ __forceinline__ float baoab_bead(const Dev<R>& d, int i, V4<R> p, const BeadPre<R>& pre,
                                            const V4<R>& f, R kick, long long step_off,
                                            V4<R>* __restrict__ pos_out, V4<R>* __restrict__ vel_out,
                                            bool chk_in, float& e2_in)
{
    V4<R> v = pre.v;
    const R im = v.w, h = d.half_dt;
    v.x += kick * im * f.x; v.y += kick * im * f.y; v.z += kick * im * f.z;
    p.x += h * v.x; p.y += h * v.y; p.z += h * v.z;
    const uint4 w = draw(d.seed, (uint32_t)pre.orig, d.ctr[CT_STEP] + step_off, ST_LANGEVIN);
    R g[3];
    gauss3<R>(w, g);
    const R sg = d.c2 * sqrt(d.kT * im);
    v.x = d.c1 * v.x + sg * g[0];
    v.y = d.c1 * v.y + sg * g[1];
    v.z = d.c1 * v.z + sg * g[2];
    p.x += h * v.x; p.y += h * v.y; p.z += h * v.z;
    pos_out[i] = p;
    vel_out[i] = v;
    // periodic images: one 32-byte record per bead, entries g | code << 29
    // (all bits set: unused; a real entry never is, g < 2^29 - 1, though the
    // z code sets the sign bit), the second half only read when the first
    // is full
    const int4 g0 = pre.g0;
    int ge[8] = { g0.x, g0.y, g0.z, g0.w, -1, -1, -1, -1 };
    if (g0.w != -1) {
        const int4 g1 = reinterpret_cast<const int4*>(d.glist)[2 * i + 1];
        ge[4] = g1.x; ge[5] = g1.y; ge[6] = g1.z; ge[7] = g1.w;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (ge[q] == -1) break;
        const int gi = ge[q] & JMASK, code = (int)((unsigned)ge[q] >> CODE_SHIFT);
        V4<R> pg = p;
        if (code & 1) pg.x -= d.L[0];
        if (code & 2) pg.y -= d.L[1];
        if (code & 4) pg.z -= d.L[2];
        pos_out[d.N + gi] = pg;
    }
    const V4<R> r = pre.xr;
    const R ex = p.x - r.x, ey = p.y - r.y, ez = p.z - r.z;
    e2_in = 0.f;
    if (chk_in) {
        const V4<R> r2 = pre.xri;
        const R fx = p.x - r2.x, fy = p.y - r2.y, fz = p.z - r2.z;
        e2_in = (float)(fx * fx + fy * fy + fz * fz);
    }
    return (float)(ex * ex + ey * ey + ez * ez);
}

// Block-wide bookkeeping of the displacements (all threads call it): beads
// beyond skin/2 (and beyond delta/2 of the inner list) are counted, and the
// block's largest squared displacement raises its slot of dmax_part.
template <typename R>
__device__ __forceinline__ void disp_stats(const Dev<R>& d, float e2, float e2_in, bool counted)
{
    __shared__ float s_m2[WG / 64];
    const unsigned long long over = __ballot(counted && e2 > (float)d.skin_half2);
    const unsigned long long over_in = __ballot(counted && e2_in > (float)d.in_half2);
    float m2 = counted ? e2 : 0.f;
    for (int o = 32; o > 0; o >>= 1) m2 = fmaxf(m2, __shfl_xor(m2, o, 64));
    if ((threadIdx.x & 63) == 0) {
        if (over) atomicAdd(&d.flags[FL_SKIN], __popcll(over));
        if (over_in) atomicAdd(&d.flags[FL_SKIN_IN], __popcll(over_in));
        s_m2[threadIdx.x >> 6] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < WG / 64; ++w) m2 = fmaxf(m2, s_m2[w]);
        // float bits of non-negative values order like integers
        atomicMax(reinterpret_cast<int*>(d.dmax_part) + blockIdx.x, __float_as_int(m2));
    }
}

// Binning for the list build.  bin_cell: the cell of a bead, its
// coordinates wrapped into [0, L) on the way.  bin_place (all 64 lanes of a
// wave call it; cell -1: no bead): beads come in slot order, which is cell
// order up to the beads that changed cell since the last rebuild, so the
// lanes form few runs of equal cells; the first lane of each run reserves
// the run's places in its cell with one atomic, and a bead's place in its
// cell (arbitrary across runs; the per-cell sort fixes the final order) is
// the reserved base plus its offset in the run.
template <typename R>
__device__ __forceinline__ int bin_cell(const Dev<R>& d, V4<R>& p)
{
    R* c[3] = { &p.x, &p.y, &p.z };
    int cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R x = *c[a];
        if (x >= d.L[a]) x -= d.L[a];        // exact (Sterbenz) for x in [L, 2L]
        else if (x < (R)0) x += d.L[a];
        if (!(x >= (R)0 && x < d.L[a])) {     // far outside (minimizer, a blown-up run)
            double xd = fmod((double)*c[a], d.Ld[a]);   // exact, in (-L, L); NaN stays NaN
            if (xd < 0.0) xd += d.Ld[a];
            x = (R)xd;
            if (!(x >= (R)0 && x < d.L[a])) x = (R)0;   // NaN, or rounded up to L
        }
        *c[a] = x;
        const int ci = (int)(x * d.inv_edge[a]);
        cc[a] = ci < 0 ? 0 : (ci >= d.nc[a] ? d.nc[a] - 1 : ci);
    }
    return (cc[0] * d.nc[1] + cc[1]) * d.nc[2] + cc[2];
}

template <typename R>
__device__ __forceinline__ void bin_place(const Dev<R>& d, int i, int cell)
{
    const int l = threadIdx.x & 63;
    const int prev = __shfl_up(cell, 1);
    const bool head = l == 0 || prev != cell;
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = l == 63 ? ~0ull : ((2ull << l) - 1);   // lanes 0..l
    const int h = 63 - __clzll((long long)(hm & upto));
    const unsigned long long above = hm & ~upto;
    int base = 0;
    if (head && cell >= 0) {
        const int len = (above ? __ffsll((long long)above) - 1 : 64) - l;
        base = atomicAdd(&d.cell_cnt[cell], len);
    }
    base = __shfl(base, h);
    if (cell >= 0) {
        d.cell_t[i] = cell;
        d.cell_pos[i] = base + l - h;
    }
}

// disp_stats when only the block's first NIW waves hold counted beads (the
// force pass that integrates: thread t < WG / lanes per bead takes bead t):
// the other waves skip it, and with one such wave there is no barrier.
template <int NIW, typename R>
__device__ __forceinline__ void disp_stats_lead(const Dev<R>& d, float e2, float e2_in, bool counted)
{
    if constexpr (NIW >= WG / 64) {
        disp_stats(d, e2, e2_in, counted);
    } else {
        __shared__ float s_m2[NIW];
        float m2 = 0.f;
        if (threadIdx.x < NIW * 64) {   // wave-uniform
            const unsigned long long over = __ballot(counted && e2 > (float)d.skin_half2);
            const unsigned long long over_in = __ballot(counted && e2_in > (float)d.in_half2);
            m2 = counted ? e2 : 0.f;
            for (int o = 32; o > 0; o >>= 1) m2 = fmaxf(m2, __shfl_xor(m2, o, 64));
            if ((threadIdx.x & 63) == 0) {
                if (over) atomicAdd(&d.flags[FL_SKIN], __popcll(over));
                if (over_in) atomicAdd(&d.flags[FL_SKIN_IN], __popcll(over_in));
                if (NIW > 1) s_m2[threadIdx.x >> 6] = m2;
            }
        }
        if constexpr (NIW > 1) {
            __syncthreads();
            if (threadIdx.x == 0)
                for (int w = 1; w < NIW; ++w) m2 = fmaxf(m2, s_m2[w]);
        }
        if (threadIdx.x == 0)
            atomicMax(reinterpret_cast<int*>(d.dmax_part) + blockIdx.x, __float_as_int(m2));
    }
}

// Entry k of slot i's neighbour list: beads are grouped by 64/lpb, and
// within a group entries are interleaved in blocks of lpb.
__host__ __device__ __forceinline__ size_t nbr_index(int i, int k, int Kcap, int lpb)
{
    const int bg = 64 / lpb;
    return (size_t)(i / bg) * ((size_t)Kcap * bg) + (size_t)(k / lpb) * 64 + (size_t)(i % bg) * lpb +
           (size_t)(k % lpb);
}

// nbr_index with power-of-two shifts: base of slot i, then + k offsets
__host__ __device__ __forceinline__ size_t nbr_base(int i, int Kcap, int lpb_shift, int bg_shift)
{
    return ((size_t)(i >> bg_shift) * (size_t)Kcap << bg_shift) +
           ((size_t)(i & ((1 << bg_shift) - 1)) << lpb_shift);
}
__host__ __device__ __forceinline__ size_t nbr_koff(int k, int lpb_shift)
{
    return ((size_t)(k >> lpb_shift) << 6) + (size_t)(k & ((1 << lpb_shift) - 1));
}

}  // namespace mbx
