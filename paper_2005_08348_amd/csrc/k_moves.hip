// k_moves.hip -- exchange moves of the paper's Theory section on the GPU.
//
// MC-MD (Eq. 1): a batch of exchange trials is drawn in counter order and
// filtered greedily (a candidate is admitted when it shares no molecule with,
// and none of its changed beads is within r_cut of a changed bead of, an
// earlier admitted candidate).  The filter is sequential by definition; here
// draws are examined in chunks: all candidates of a chunk are drawn, located
// and checked against the trials admitted so far in parallel (one wave
// each), conflicts between them are listed through a spatial hash, and the
// lexicographically-first admission is resolved by parallel rounds in one
// work-group (a candidate is in once every earlier conflicting candidate is
// out, out as soon as one is in), which reproduces the sequential order
// exactly.  Each admitted trial's dU = U(after) - U(before)
// is the float64 sum of pair-energy changes over its changed beads'
// neighbour lists.
//
// MDAS (Eqs. 2-3): the selected pairs' changed beads are marked with their
// end-state class; the force difference F_B - F_A and dU = U_B - U_A come from
// the beads whose pair terms change (the changed beads and their
// neighbours), so F(lambda) = F_A + lambda (F_B - F_A) and the work
// increments cost no extra force evaluation.
#include "membx_dev.h"

namespace mbx {

template <typename R> __device__ __forceinline__ R rsq_m(R x);
template <> __device__ __forceinline__ float rsq_m<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsq_m<double>(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ double dwave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// float64 minimum-image squared distance (rint image, no contraction)
template <typename R>
__device__ __forceinline__ double mi_dist2(const Dev<R>& d, const double* a, const double* b)
{
#pragma clang fp contract(off)
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double t = a[k] - b[k];
        t -= d.Ld[k] * rint(t / d.Ld[k]);
        r2 = (k == 0) ? t * t : r2 + t * t;
    }
    return r2;
}

template <typename R>
__device__ __forceinline__ int hash_cell(const Dev<R>& d, const Mv& m, const double* p, int c[3])
{
    for (int k = 0; k < 3; ++k) {
        int q = (int)floor(p[k] * m.hinv[k]);
        q %= m.hnc[k];
        if (q < 0) q += m.hnc[k];
        c[k] = q;
    }
    return (c[0] * m.hnc[1] + c[1]) * m.hnc[2] + c[2];
}

// Bucket word {epoch:32, key:24, count:8}.  Words and entries that the
// same kernel may have written are read with device-coherent atomic loads:
// inserts land at L2 through atomics, which a plain load through the CU's L1
// could miss.
typedef unsigned long long u64;
__device__ __forceinline__ u64 hw_make(unsigned ep, unsigned key, unsigned n)
{
    return ((u64)ep << 32) | ((u64)(key & 0xffffffu) << 8) | (u64)n;
}
__device__ __forceinline__ unsigned hw_ep(u64 w) { return (unsigned)(w >> 32); }
__device__ __forceinline__ unsigned hw_key(u64 w) { return (unsigned)(w >> 8) & 0xffffffu; }
__device__ __forceinline__ unsigned hw_n(u64 w) { return (unsigned)(w & 0xffu); }
__device__ __forceinline__ unsigned hhash(unsigned key) { return key * 2654435761u; }
__device__ __forceinline__ u64 hw_load(const u64* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_coh(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// COH: device-coherent (the kernel itself may have written the word);
// otherwise a plain load, for data written by earlier launches only (a
// kernel boundary makes it visible, and the load may hit in the L2)
template <bool COH, typename T>
__device__ __forceinline__ T ld_sel(const T* p)
{
    if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}

__device__ __forceinline__ void hb_insert(u64* word, int* ent, int mask, unsigned key, int e,
                                          unsigned ep)
{
    key &= 0xffffffu;
    unsigned h = hhash(key) & (unsigned)mask;
    u64 w = hw_load(&word[h]);
    while (true) {
        if (hw_ep(w) != ep) {
            u64 got = atomicCAS(&word[h], w, hw_make(ep, key, 1));
            if (got == w) { __hip_atomic_store(&ent[h * HBW], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); return; }
            w = got;
            continue;
        }
        if (hw_key(w) == key && hw_n(w) < HBW) {
            u64 got = atomicCAS(&word[h], w, w + 1);
            if (got == w) {
                __hip_atomic_store(&ent[h * HBW + hw_n(w)], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            w = got;
            continue;
        }
        h = (h + 1) & (unsigned)mask;
        w = hw_load(&word[h]);
    }
}

// Key of neighbour cell o27 (0..26) of the cell holding p.
template <typename R>
__device__ __forceinline__ unsigned nbr_cell_key(const Dev<R>& d, const Mv& m, const double* p,
                                                 int o27)
{
    int c[3];
    hash_cell(d, m, p, c);
    const int cx = (c[0] + o27 / 9 - 1 + m.hnc[0]) % m.hnc[0];
    const int cy = (c[1] + (o27 / 3) % 3 - 1 + m.hnc[1]) % m.hnc[1];
    const int cz = (c[2] + o27 % 3 - 1 + m.hnc[2]) % m.hnc[2];
    return (unsigned)((cx * m.hnc[1] + cy) * m.hnc[2] + cz);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int ln = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (ln >= o) v += u;
    }
    return v;
}

// ------------------------------------------------------------------------
// Candidate selection.  mode 0: exchange batch (random stream 1, counter =
// batch, spatial filter); mode 1: MDAS pairs (stream 3, counter = cycle,
// distinct molecules only).  The trials admitted are the greedy filter in
// draw order: a draw is admitted when neither molecule is used by an earlier
// admitted trial and (mode 0) none of its changed beads lies within r_cut
// (float64 minimum image) of an admitted trial's changed bead.  Draws are
// examined in chunks; a chunk's admissions are the lexicographically-first
// independent set of its conflict graph restricted to candidates free of the
// trials admitted before the chunk, which is what the sequential filter
// admits.  Chunk sizes only change the cost, never the result.

// One wave per candidate: draw, partner, changed beads.  Returns the flag
// (0 live, 1 no valid trial, 2 molecule already used) and fills X, Y, nb;
// lane q < nb returns bead q's id, class and position.
template <bool COH, typename R>
__device__ __forceinline__ int sel_candidate(const Dev<R>& d, const Mv& m, int dd, long long ctrv,
                                             unsigned stream, int stamp, int& X, int& Y, int& nb,
                                             int& bead, int& cls, double p[3])
{
    X = -1; Y = -1; nb = 0;
    const int ln = threadIdx.x & 63;
    if (m.n_sw <= 0) return 1;
    const uint4 w = draw(d.seed, (uint32_t)dd, ctrv, stream);
    X = m.sw_list[pick(w.x, (uint32_t)m.n_sw)];
    const int kx = ld_sel<COH>(d.mol_kind + X);
    const int f = m.fam_of_kind[kx];
    if (m.xmode == 0) {
        const int nf = m.fam_off[f + 1] - m.fam_off[f];
        const int noth = nf - m.kcnt[kx * m.fam_stride + nf];
        if (noth <= 0) return 1;
        Y = m.others[kx * m.fam_stride + pick(w.y, (uint32_t)noth)];
    } else if (m.xmode == 1) {   // another kind, same region
        const int r = m.region[X];
        const int nr = m.reg_off[2 * f + r + 1] - m.reg_off[2 * f + r];
        const int base = (kx * 2 + r) * m.fam_stride;
        const int noth = nr - m.kcnt_r[base + nr];
        if (noth <= 0) return 1;
        Y = m.others_r[base + pick(w.y, (uint32_t)noth)];
    } else {                     // any member of the other region
        const int r = 1 - m.region[X];
        const int o0 = m.reg_off[2 * f + r], nr = m.reg_off[2 * f + r + 1] - o0;
        if (nr <= 0) return 1;
        Y = m.reg_mem[o0 + pick(w.y, (uint32_t)nr)];
    }
    const int ky = ld_sel<COH>(d.mol_kind + Y);
    const int flag = (ld_sel<COH>(m.used + X) == stamp || ld_sel<COH>(m.used + Y) == stamp) ? 2 : 0;
    const int nch = m.chg_n[kx * d.nk + ky];
    nb = 2 * nch;
    if (ln < nb) {
        const int* loc = m.chg_loc + (kx * d.nk + ky) * MAXCH;
        const bool first = ln < nch;
        const int l = loc[first ? ln : ln - nch];
        bead = (first ? d.mol_first[X] : d.mol_first[Y]) + l;
        cls = d.kcls[d.kbead_off[first ? ky : kx] + l];
        const V4<R> q = d.posq[d.inv[bead]];
        p[0] = (double)q.x; p[1] = (double)q.y; p[2] = (double)q.z;
    }
    return flag;
}

// Wave-wide: does any changed bead (positions in sp[3*q], q < nb) lie within
// r_cut of a changed bead of the trials admitted so far (table ab, epoch
// stamp)?
template <bool COH, typename R>
__device__ __forceinline__ bool sel_hits_admitted(const Dev<R>& d, const Mv& m, const double* sp,
                                                  int nb, unsigned stamp)
{
    const int ln = threadIdx.x & 63;
    bool hit = false;
    for (int it = ln; it < nb * 27; it += 64) {
        const int q = it / 27, o27 = it - q * 27;
        const double* p = sp + 3 * q;
        const unsigned key = nbr_cell_key(d, m, p, o27);
        unsigned h = hhash(key) & (unsigned)m.ab_mask;
        u64 w = ld_sel<COH>(&m.ab_word[h]);
        while (!hit && hw_ep(w) == stamp) {
            if (hw_key(w) == key)
                for (unsigned s = 0; s < hw_n(w) && s < HBW; ++s) {
                    const int e = ld_sel<COH>(m.ab_ent + h * HBW + s);
                    double r[3];
                    for (int k = 0; k < 3; ++k) r[k] = ld_sel<COH>(m.r_pos + 3 * e + k);
                    if (mi_dist2(d, p, r) < d.rc2d) hit = true;
                }
            h = (h + 1) & (unsigned)m.ab_mask;
            w = ld_sel<COH>(&m.ab_word[h]);
        }
    }
    return __ballot(hit) != 0;
}

// Draw the chunk's candidates (one wave each), set them aside when a
// molecule is used or (mode 0) a changed bead is within r_cut of an admitted
// trial, and hash the live ones (cells of their changed beads, molecules).
template <typename R>
__global__ __launch_bounds__(256) void k_sel_draw(Dev<R> d, Mv m, int draw_cap, int mode, int ck)
{
    __shared__ double s_pos[4][MAXMC * 3];
    if (m.sel[SEL_DONE]) return;
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
    const int MC = m.maxcht;
    const unsigned ep = (unsigned)m.sel[SEL_EPC];
    const int stamp = m.sel[SEL_STAMP];
    const int dd = m.sel[SEL_NEXT] + t;
    const long long ctrv = d.ctr[mode == 0 ? CT_BATCH : CT_CYCLE];
    const unsigned stream = mode == 0 ? ST_SWAP_DRAW : ST_MDAS_SELECT;
    int flag = 1, X = -1, Y = -1, nb = 0, bead = -1, cls = 0;
    double p[3] = {0.0, 0.0, 0.0};
    if (t < ck && dd < draw_cap)
        flag = sel_candidate<false>(d, m, dd, ctrv, stream, stamp, X, Y, nb, bead, cls, p);
    if (flag != 1 && ln < nb) {
        const int e = t * MC + ln;
        m.c_bead[e] = bead;
        m.c_cls[e] = cls;
        for (int k = 0; k < 3; ++k) { m.c_pos[3 * e + k] = p[k]; s_pos[wv][3 * ln + k] = p[k]; }
    }
    __syncthreads();
    if (flag == 0 && mode == 0 && m.sel[SEL_ADM] > 0 &&
        sel_hits_admitted<false>(d, m, s_pos[wv], nb, (unsigned)stamp))
        flag = 2;
    if (flag == 0) {
        if (mode == 0 && ln < nb) {
            int c[3];
            hb_insert(m.hb_word, m.hb_ent, m.hb_mask, (unsigned)hash_cell(d, m, p, c), t * MC + ln, ep);
        }
        if (ln == 62) hb_insert(m.mb_word, m.mb_ent, m.mb_mask, (unsigned)X, 2 * t, ep);
        if (ln == 63) hb_insert(m.mb_word, m.mb_ent, m.mb_mask, (unsigned)Y, 2 * t + 1, ep);
    }
    if (ln == 0 && t < ck) {
        m.c_flag[t] = flag;
        m.c_x[t] = X;
        m.c_y[t] = Y;
        m.c_nb[t] = nb;
        m.c_conf_n[t] = 0;
    }
}

// Conflict lists (one wave per live candidate): the earlier live candidates
// of the chunk that share a molecule with it or (mode 0) have a changed bead
// within r_cut of one of its own, ascending, at most SEL_CAPC listed (the
// count is exact).
template <typename R>
__global__ __launch_bounds__(256) void k_sel_conf(Dev<R> d, Mv m, int mode, int ck)
{
    __shared__ unsigned s_bits[4][SEL_CMAX / 32];
    if (m.sel[SEL_DONE]) return;
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
    const int MC = m.maxcht;
    const bool act = t < ck && m.c_flag[t] == 0;
    const unsigned ep = (unsigned)m.sel[SEL_EPC];
    const int nw = (t + 31) >> 5;
    unsigned* bits = s_bits[wv];
    if (act)
        for (int i = ln; i < nw; i += 64) bits[i] = 0u;
    __syncthreads();
    if (act) {
        const int nb = m.c_nb[t];
        const int nsp = mode == 0 ? nb * 27 : 0;
        for (int it = ln; it < nsp + 2; it += 64) {
            if (it < nsp) {
                const int q = it / 27, o27 = it - q * 27;
                const double* pq = m.c_pos + 3 * (t * MC + q);
                const double p[3] = {pq[0], pq[1], pq[2]};
                const unsigned key = nbr_cell_key(d, m, p, o27);
                unsigned h = hhash(key) & (unsigned)m.hb_mask;
                u64 w = m.hb_word[h];
                while (hw_ep(w) == ep) {
                    if (hw_key(w) == key)
                        for (unsigned s = 0; s < hw_n(w) && s < HBW; ++s) {
                            const int e = m.hb_ent[h * HBW + s];
                            const int o = e / MC;
                            if (o < t && mi_dist2(d, p, m.c_pos + 3 * e) < d.rc2d)
                                atomicOr(&bits[o >> 5], 1u << (o & 31));
                        }
                    h = (h + 1) & (unsigned)m.hb_mask;
                    w = m.hb_word[h];
                }
            } else {
                const unsigned key = (unsigned)(it == nsp ? m.c_x[t] : m.c_y[t]) & 0xffffffu;
                unsigned h = hhash(key) & (unsigned)m.mb_mask;
                u64 w = m.mb_word[h];
                while (hw_ep(w) == ep) {
                    if (hw_key(w) == key)
                        for (unsigned s = 0; s < hw_n(w) && s < HBW; ++s) {
                            const int o = m.mb_ent[h * HBW + s] >> 1;
                            if (o < t) atomicOr(&bits[o >> 5], 1u << (o & 31));
                        }
                    h = (h + 1) & (unsigned)m.mb_mask;
                    w = m.mb_word[h];
                }
            }
        }
    }
    __syncthreads();
    if (act) {
        int total = 0;
        for (int i0 = 0; i0 < nw; i0 += 64) {
            const int i = i0 + ln;
            unsigned b = i < nw ? bits[i] : 0u;
            const int c = __popc(b);
            const int incl = wave_incl_scan(c);
            int pos = total + incl - c;
            while (b) {
                const int bit = __ffs(b) - 1;
                b &= b - 1;
                if (pos < SEL_CAPC) m.c_conf[t * SEL_CAPC + pos] = i * 32 + bit;
                ++pos;
            }
            total += __shfl(incl, 63, 64);
        }
        if (ln == 0) m.c_conf_n[t] = total;
    }
}

// Admit candidate t as trial a (caller: the lanes of one wave).
template <typename R>
__device__ __forceinline__ void sel_admit(const Dev<R>& d, const Mv& m, int mode, int a, int draw_idx,
                                          int X, int Y, int nb, const int* bead, const int* cls,
                                          const double* pos, int lane0, int nlanes, int stamp)
{
    const int MC = m.maxcht;
    for (int q = lane0; q < nb; q += nlanes) {
        m.r_bead[a * MC + q] = bead[q];
        m.r_cls[a * MC + q] = cls[q];
        for (int k = 0; k < 3; ++k)
            __hip_atomic_store(m.r_pos + 3 * (a * MC + q) + k, pos[3 * q + k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (mode == 0) {
            int c[3];
            hb_insert(m.ab_word, m.ab_ent, m.ab_mask, (unsigned)hash_cell(d, m, pos + 3 * q, c),
                      a * MC + q, (unsigned)stamp);
        }
    }
    if (lane0 == 0) {
        m.r_draw[a] = draw_idx;
        m.r_x[a] = X;
        m.r_y[a] = Y;
        m.r_nb[a] = nb;
        __hip_atomic_store(m.used + X, stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(m.used + Y, stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Exclusive prefix over the 1024 threads of a work-group (wave scans, then
// the 16 wave totals); *total (LDS) receives the sum.  Contains barriers:
// every thread calls it.
__device__ __forceinline__ int block1024_excl_scan(int v, int* s_w, int* total)
{
    const int tid = threadIdx.x, ln = tid & 63, w = tid >> 6;
    const int incl = wave_incl_scan(v);
    if (ln == 63) s_w[w] = incl;
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) base += q < w ? s_w[q] : 0;
    if (tid == 1023) *total = base + incl;
    __syncthreads();
    return base + incl - v;
}

// Resolve the chunk (one work-group): the lexicographically-first admission
// by parallel rounds over the conflict lists held in LDS (in once every
// earlier conflicting candidate is out, out as soon as one is in), then the
// admitted candidates in draw order up to the number still wanted.  A
// candidate whose list is incomplete, or does not fit, ends the chunk there:
// the next chunk starts with its draw.
static_assert(SEL_CMAX <= SEL_LDS, "the admitted list of a chunk reuses the conflict-list LDS");
static_assert(4 * SEL_C0 <= SEL_CMAX && SEL_C0 % 4 == 0, "chunk sizes of launch_select");
template <typename R>
__global__ __launch_bounds__(1024) void k_sel_resolve(Dev<R> d, Mv m, int n_want, int draw_cap,
                                                      int mode, int ck)
{
    constexpr int PER = SEL_CMAX / 1024;
    __shared__ unsigned char stb[2][SEL_CMAX];   // status, double-buffered by round
    __shared__ short lst[SEL_LDS];
    __shared__ int s_red[64];
    __shared__ int s_trunc, s_chg[3], s_stop;
    if (m.sel[SEL_DONE]) return;
    const int tid = threadIdx.x;
    const int per = (ck + 1023) / 1024;
    const int t0 = tid * per;
    const int MC = m.maxcht;
    const int base = m.sel[SEL_NEXT];
    const int adm = m.sel[SEL_ADM];
    const int stamp = m.sel[SEL_STAMP];
    if (tid == 0) { s_trunc = ck; s_stop = -1; s_chg[0] = 0; s_chg[1] = 0; s_chg[2] = 0; }
    // per-thread candidates t0 .. t0 + per - 1 (register arrays, loops unrolled)
    int cnt[PER], off[PER], nst[PER], skip[PER];
    int mysum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = t0 + k;
        cnt[k] = 0;
        if (k < per && t < ck && m.c_flag[t] == 0) cnt[k] = m.c_conf_n[t];
        mysum += cnt[k] < SEL_CAPC ? cnt[k] : SEL_CAPC;
    }
    // exclusive prefix of the list lengths
    int run = block1024_excl_scan(mysum, s_red, s_red + 16);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        off[k] = run;
        if (k < per && (cnt[k] > SEL_CAPC || run + cnt[k] > SEL_LDS)) atomicMin(&s_trunc, t0 + k);
        run += cnt[k] < SEL_CAPC ? cnt[k] : SEL_CAPC;
    }
    __syncthreads();
    const int trunc = s_trunc;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = t0 + k;
        const bool live = k < per && t < trunc && m.c_flag[t] == 0;
        if (!live) cnt[k] = 0;
        // the list in 16-byte reads, 16 entries per round trip (a row holds
        // SEL_CAPC entries and starts on a 256-byte boundary)
        const int4* row = reinterpret_cast<const int4*>(m.c_conf + (size_t)t * SEL_CAPC);
        for (int j0 = 0; j0 < cnt[k]; j0 += 16) {
            int4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                v[u] = j0 + 4 * u < cnt[k] ? row[(j0 >> 2) + u] : make_int4(0, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e[4] = { v[u].x, v[u].y, v[u].z, v[u].w };
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int j = j0 + 4 * u + c;
                    if (j < cnt[k]) lst[off[k] + j] = (short)e[c];
                }
            }
        }
        nst[k] = live ? 0 : 2;
        skip[k] = 0;
        if (k < per) stb[0][t] = (unsigned char)nst[k];
    }
    __syncthreads();
    // Rounds with one barrier each: round r reads the status buffer r & 1 and
    // writes every own status to the other, which nobody reads before the
    // barrier; the change flag of round r is s_chg[r % 3], cleared two rounds
    // ahead (its last readers passed a barrier since).
    for (int r = 0;; ++r) {
        const unsigned char* cur = stb[r & 1];
        unsigned char* nxt = stb[(r + 1) & 1];
        if (tid == 0) s_chg[(r + 1) % 3] = 0;
        bool changed = false;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (nst[k] == 0) {
                // scan from the first entry not yet known to be out, eight
                // independent LDS reads at a time; entries decided out at
                // the head are skipped in later rounds
                bool anyin = false, anyund = false;
                int head = skip[k];
                for (int j0 = skip[k]; j0 < cnt[k]; j0 += 8) {
                    short e[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) e[u] = j0 + u < cnt[k] ? lst[off[k] + j0 + u] : (short)-1;
                    unsigned char v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = e[u] >= 0 ? cur[e[u]] : (unsigned char)2;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        anyin |= (v[u] == 1);
                        anyund |= (v[u] == 0);
                        if (head == j0 + u && v[u] == 2) ++head;
                    }
                }
                skip[k] = head;
                const int v = anyin ? 2 : (anyund ? 0 : 1);
                if (v != 0) { nst[k] = v; changed = true; }
            }
            if (k < per) nxt[t0 + k] = (unsigned char)nst[k];
        }
        if (changed) s_chg[r % 3] = 1;
        __syncthreads();
        if (!s_chg[r % 3]) break;
    }
    // admitted candidates in draw order (rank), listed in LDS (the conflict
    // lists are no longer read), then written out one (trial, changed bead)
    // per thread: the hash inserts of a trial's beads run side by side
    int nin = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) nin += (k < per && nst[k] == 1) ? 1 : 0;
    int rank = block1024_excl_scan(nin, s_red + 32, s_red + 48);
    const int total = s_red[48];
    const int need = n_want - adm;
    const int nadm_c = total < need ? total : need;   // admitted in this chunk
    short* adm_t = lst;                               // [nadm_c] <= ck <= SEL_LDS
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = t0 + k;
        if (k < per && nst[k] == 1) {
            if (rank < need) {
                adm_t[rank] = (short)t;
                if (rank == need - 1) s_stop = t;
            }
            ++rank;
        }
    }
    __syncthreads();
    for (int w = tid; w < nadm_c * MC; w += 1024) {
        const int a = w / MC, q = w - a * MC, t = adm_t[a];
        sel_admit(d, m, mode, adm + a, base + t, m.c_x[t], m.c_y[t], m.c_nb[t], m.c_bead + t * MC,
                  m.c_cls + t * MC, m.c_pos + 3 * t * MC, q, MC, stamp);
    }
    __syncthreads();
    if (tid == 0) {
        const int nadm = adm + (total < need ? total : need);
        const int next = s_stop >= 0 ? base + s_stop + 1 : base + trunc;
        m.sel[SEL_ADM] = nadm;
        m.sel[SEL_NEXT] = next;
        m.sel[SEL_DONE] = (nadm >= n_want || next >= draw_cap) ? 1 : 0;
        m.sel[SEL_EPC] = m.sel[SEL_EPC] + 1;
        m.r_n[0] = nadm;
        m.r_n[1] = next < draw_cap ? next : draw_cap;
    }
}

// Finish the selection one draw at a time (one wave) when the chunks did not
// reach the end.
template <typename R>
__global__ __launch_bounds__(64) void k_sel_tail(Dev<R> d, Mv m, int n_want, int draw_cap, int mode)
{
    __shared__ double s_pos[MAXMC * 3];
    __shared__ int s_bead[MAXMC], s_cls[MAXMC];
    if (m.sel[SEL_DONE]) return;
    const int ln = threadIdx.x;
    const int stamp = m.sel[SEL_STAMP];
    const long long ctrv = d.ctr[mode == 0 ? CT_BATCH : CT_CYCLE];
    const unsigned stream = mode == 0 ? ST_SWAP_DRAW : ST_MDAS_SELECT;
    int adm = m.sel[SEL_ADM];
    int dd = m.sel[SEL_NEXT];
    for (; dd < draw_cap && adm < n_want; ++dd) {
        int X, Y, nb, bead = -1, cls = 0;
        double p[3] = {0.0, 0.0, 0.0};
        int flag = sel_candidate<true>(d, m, dd, ctrv, stream, stamp, X, Y, nb, bead, cls, p);
        if (flag != 1 && ln < nb) {
            s_bead[ln] = bead;
            s_cls[ln] = cls;
            for (int k = 0; k < 3; ++k) s_pos[3 * ln + k] = p[k];
        }
        __syncthreads();
        if (flag == 0 && mode == 0 && adm > 0 && sel_hits_admitted<true>(d, m, s_pos, nb, (unsigned)stamp))
            flag = 2;
        if (flag == 0) {
            sel_admit(d, m, mode, adm, dd, X, Y, nb, s_bead, s_cls, s_pos, ln, 64, stamp);
            ++adm;
        }
        __threadfence();
        __syncthreads();
    }
    if (ln == 0) {
        m.sel[SEL_ADM] = adm;
        m.sel[SEL_NEXT] = dd;
        m.sel[SEL_DONE] = 1;
        m.r_n[0] = adm;
        m.r_n[1] = dd < draw_cap ? dd : draw_cap;
    }
}

// Start a selection: fresh stamp (molecules used, admitted-bead table) and
// chunk epoch.
__global__ void k_sel_init(Mv m, int n_want)
{
    const int c = m.sel[SEL_EPC];
    m.sel[SEL_STAMP] = c + 1;
    m.sel[SEL_EPC] = c + 2;
    m.sel[SEL_ADM] = 0;
    m.sel[SEL_NEXT] = 0;
    m.sel[SEL_DONE] = n_want <= 0 ? 1 : 0;
    m.r_n[0] = 0;
    m.r_n[1] = 0;
}

// Mark the changed beads of the admitted trials (tag = trial for exchange
// batches, 0 for MDAS) with their new class.
template <typename R>
__global__ void k_mark(Dev<R> d, Mv m, int mode)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) *m.aff_n = 0;   // the affected set of these trials starts empty
    int MC = m.maxcht;
    int a = e / MC, q = e % MC;
    if (a >= m.r_n[0] || q >= m.r_nb[a]) return;
    int s = d.inv[m.r_bead[a * MC + q]];
    d.alch[s] = m.r_cls[a * MC + q] | ((mode == 0 ? a : 0) << 8);
}

__device__ __forceinline__ int owner_of(const int* ghost_owner, int N, int j)
{
    return j < N ? j : ghost_owner[j - N];
}

// Pair-energy change summed over one changed bead's neighbour list (one wave
// per changed bead).  Pairs between two changed beads of the same trial are
// visited from both ends and weighted 1/2.
template <typename R>
__global__ __launch_bounds__(64) void k_du_bead(Dev<R> d, Mv m)
{
    const int e = blockIdx.x, lane = threadIdx.x;
    const int MC = m.maxcht;
    const int a = e / MC, q = e % MC;
    if (a >= m.r_n[0] || q >= m.r_nb[a]) {
        if (lane == 0) m.du_bead[e] = 0.0;
        return;
    }
    const int i = d.inv[m.r_bead[a * MC + q]];
    const V4<R> pi = d.posq[i];
    const int ci = cls_of<R>(pi.w);
    const int mk = d.alch[i];
    const int ci2 = mk & 0xff, tag = mk >> 8;
    const int n1 = d.ncnt[i];
    double du = 0.0;
    for (int k = lane; k < n1; k += 64) {
        int en = d.nbr[nbr_index(i, k, d.Kcap, d.lpb)];
        int j = en & JMASK, code = (int)((unsigned)en >> CODE_SHIFT);
        V4<R> pj = d.posq[j];
        int o = owner_of(d.ghost_owner, d.N, j);
        int cj = cls_of<R>(d.posq[o].w);
        int mj = d.alch[o];
        int cj2 = cj;
        double wgt = 1.0;
        if (mj >= 0 && (mj >> 8) == tag) { cj2 = mj & 0xff; wgt = 0.5; }
        R xs = (code & 1) ? pi.x - d.L[0] : pi.x;
        R ys = (code & 2) ? pi.y - d.L[1] : pi.y;
        R zs = (code & 4) ? pi.z - d.L[2] : pi.z;
        R dx = xs - pj.x, dy = ys - pj.y, dz = zs - pj.z;
        R r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < d.rc2) {
            R rinv = rsq_m<R>(r2), rinv2 = rinv * rinv, rinv6 = rinv2 * rinv2 * rinv2;
            R g = rinv + d.krf * r2 - d.crf;
            V4<R> p1 = d.tabE[ci2 * MAXCLS + cj2], p0 = d.tabE[ci * MAXCLS + cj];
            R v1 = (p1.y * rinv6 - p1.x) * rinv6 - p1.w + p1.z * g;
            R v0 = (p0.y * rinv6 - p0.x) * rinv6 - p0.w + p0.z * g;
            du += wgt * ((double)v1 - (double)v0);
        }
    }
    du = dwave_sum(du);
    if (lane == 0) m.du_bead[e] = du;
}

// Per-trial dU (fixed order), Metropolis test u < exp(-dU/kT) (Eq. 1).
template <typename R>
__global__ void k_trial_accept(Dev<R> d, Mv m)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m.r_n[0]) return;
    int MC = m.maxcht;
    double du = 0.0;
    for (int q = 0; q < m.r_nb[a]; ++q) du += m.du_bead[a * MC + q];
    du += m.du_bond[a];
    uint4 w = draw(d.seed, (uint32_t)m.r_draw[a], d.ctr[CT_BATCH], ST_SWAP_ACCEPT);
    double u = u53(w.x, w.y);
    int acc = u < exp(-du / d.kTd);
    m.r_du[a] = du;
    m.r_u[a] = u;
    m.r_acc[a] = acc;
    // a rejected trial's marks are cleared here; the accepted ones by the commit
    if (!acc)
        for (int q = 0; q < m.r_nb[a]; ++q) d.alch[d.inv[m.r_bead[a * MC + q]]] = -1;
}

// Total dU over every admitted change (MDAS: U_B - U_A at the current x).
template <typename R>
__global__ __launch_bounds__(64) void k_du_total(Dev<R> d, Mv m, double* out)
{
    // one wave: lane a sums trial a's bead terms and bonded change in bead
    // order (the trials' loads all in flight), then lane 0 adds the trials
    // in order, 64 at a time
    __shared__ double part[64];
    const int ln = threadIdx.x, MC = m.maxcht, n = m.r_n[0];
    double s = 0.0;
    for (int a0 = 0; a0 < n; a0 += 64) {
        const int a = a0 + ln;
        double p = 0.0;
        if (a < n) {
            const int nb = m.r_nb[a];
            for (int q = 0; q < nb; ++q) p += m.du_bead[a * MC + q];
            p += m.du_bond[a];
        }
        part[ln] = p;
        __syncthreads();
        if (ln == 0)
            for (int k = 0; k < 64 && a0 + k < n; ++k) s += part[k];
        __syncthreads();
    }
    if (ln == 0) *out = s;
}

// Affected set: the marked beads and every bead in their neighbour lists.
template <typename R>
__global__ __launch_bounds__(64) void k_aff_mark(Dev<R> d, Mv m, int only_accepted)
{
    const int e = blockIdx.x, lane = threadIdx.x;
    const int MC = m.maxcht;
    const int a = e / MC, q = e % MC;
    if (a >= m.r_n[0] || q >= m.r_nb[a]) return;
    if (only_accepted && !m.r_acc[a]) return;
    const int i = d.inv[m.r_bead[a * MC + q]];
    const int n1 = d.ncnt[i];
    for (int k = lane - 1; k < n1; k += 64) {
        int s = (k < 0) ? i : owner_of(d.ghost_owner, d.N, d.nbr[nbr_index(i, k, d.Kcap, d.lpb)] & JMASK);
        if (atomicExch(&m.aff_flag[s], 1) == 0) {
            int idx = atomicAdd(m.aff_n, 1);
            if (idx < m.aff_cap) m.aff_list[idx] = s;
            else atomicOr(&d.flags[FL_AFF_OVF], 1);
        }
    }
}

template <typename R>
__global__ void k_aff_clear(Dev<R> d, Mv m)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int n = min(*m.aff_n, m.aff_cap);
    if (k < n) m.aff_flag[m.aff_list[k]] = 0;
}

__global__ void k_zero1(int* p) { *p = 0; }

// Force difference F_new - F_old on each affected bead (LPB = 8 lanes per
// bead); every marked bead takes its new class.  scale: added to the stored
// force (1 for an applied exchange, lambda for MDAS); the difference itself
// is kept in dfrc for later lambda increments.
template <typename R>
__global__ __launch_bounds__(WG) void k_dforce(Dev<R> d, Mv m, R scale)
{
    const int gid = blockIdx.x * WG + threadIdx.x;
    const int k0 = gid >> 3, s = gid & 7;
    const int na = min(*m.aff_n, m.aff_cap);
    const bool valid = k0 < na;
    const int i = valid ? m.aff_list[k0] : 0;
    R fx = 0, fy = 0, fz = 0;
    if (valid) {
        const V4<R> pi = d.posq[i];
        const int ci = cls_of<R>(pi.w);
        const int mk = d.alch[i];
        const int ci2 = mk >= 0 ? (mk & 0xff) : ci;
        const int n1 = d.ncnt[i];
        // KB entries per lane at a time: entries, then owners, then marks,
        // each with all its loads in flight (most pairs have no mark and
        // stop there)
        constexpr int KB = 4;
        for (int kb = s; kb < n1; kb += 8 * KB) {
            int ent[KB], own[KB], mrk[KB];
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                const int k = kb + 8 * b;
                ent[b] = k < n1 ? d.nbr[nbr_index(i, k, d.Kcap, d.lpb)] : 0;
            }
#pragma unroll
            for (int b = 0; b < KB; ++b)
                own[b] = kb + 8 * b < n1 ? owner_of(d.ghost_owner, d.N, ent[b] & JMASK) : 0;
#pragma unroll
            for (int b = 0; b < KB; ++b) mrk[b] = kb + 8 * b < n1 ? d.alch[own[b]] : -1;
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                if (kb + 8 * b >= n1) continue;
                const int en = ent[b], o = own[b], mj = mrk[b];
                int j = en & JMASK, code = (int)((unsigned)en >> CODE_SHIFT);
                if (mk < 0 && mj < 0) continue;
                V4<R> pj = d.posq[j];
                int cj = cls_of<R>(d.posq[o].w);
                int cj2 = mj >= 0 ? (mj & 0xff) : cj;
                R xs = (code & 1) ? pi.x - d.L[0] : pi.x;
                R ys = (code & 2) ? pi.y - d.L[1] : pi.y;
                R zs = (code & 4) ? pi.z - d.L[2] : pi.z;
                R dx = xs - pj.x, dy = ys - pj.y, dz = zs - pj.z;
                R r2 = dx * dx + dy * dy + dz * dz;
                if (!(r2 < d.rc2)) continue;
                R rinv = rsq_m<R>(r2), rinv2 = rinv * rinv, rinv6 = rinv2 * rinv2 * rinv2;
                V4<R> p1 = d.tabF[ci2 * MAXCLS + cj2], p0 = d.tabF[ci * MAXCLS + cj];
                R f1 = (p1.y * rinv6 - p1.x) * (rinv6 * rinv2) + (p1.z * (rinv * rinv2) - p1.w);
                R f0 = (p0.y * rinv6 - p0.x) * (rinv6 * rinv2) + (p0.z * (rinv * rinv2) - p0.w);
                R fs = f1 - f0;
                fx += fs * dx; fy += fs * dy; fz += fs * dz;
            }
        }
    }
#pragma unroll
    for (int q = 4; q >= 1; q >>= 1) {
        fx += __shfl_xor(fx, q);
        fy += __shfl_xor(fy, q);
        fz += __shfl_xor(fz, q);
    }
    if (valid && s == 0) {
        d.dfrc[i] = V4<R>{ fx, fy, fz, (R)0 };
        V4<R> f = d.frc[i];
        f.x += scale * fx; f.y += scale * fy; f.z += scale * fz;
        d.frc[i] = f;
    }
}

// ------------------------------------------------ soft-core lambda path
// Eq. 4 as the MDAS path (float64 throughout): a pair with a changed bead
// takes the A-state LJ at mu = 1 - lambda and the B-state LJ at mu =
// lambda, each mu (c12 / s^6 - c6 / s^3) with s = r^2 + delta (1 - mu),
// shifted to zero at the cutoff, plus the reaction field of the
// interpolated charge product (tabE rows: c6, c12, f q_i q_j / eps_r).  At
// lambda = 0 this is the plain A pair, so the force pass (A classes) plus
// F_sc(lambda) - F_sc(0) on the affected beads is the force at lambda.
__device__ __forceinline__ void sc_lj_d(double c6, double c12, double r2, double mu, double delta,
                                        double rc2, double& v, double& fs)
{
    const double sh = delta * (1.0 - mu);
    const double s3 = r2 + sh, i3 = 1.0 / (s3 * s3 * s3);
    const double c3 = rc2 + sh, ic3 = 1.0 / (c3 * c3 * c3);
    v = mu * (c12 * i3 * i3 - c6 * i3) - mu * (c12 * ic3 * ic3 - c6 * ic3);
    fs = mu * (12.0 * c12 * i3 * i3 - 6.0 * c6 * i3) / s3;
}

template <typename R>
__device__ __forceinline__ void sc_pair_d(const Dev<R>& d, int ci, int cj, int ci2, int cj2, double r2,
                                          double lam, double delta, double& v, double& fs)
{
    const V4<R> ea = d.tabE[ci * MAXCLS + cj], eb = d.tabE[ci2 * MAXCLS + cj2];
    double va, fa, vb, fb;
    sc_lj_d((double)ea.x, (double)ea.y, r2, 1.0 - lam, delta, d.rc2d, va, fa);
    sc_lj_d((double)eb.x, (double)eb.y, r2, lam, delta, d.rc2d, vb, fb);
    const double qq = (1.0 - lam) * (double)ea.z + lam * (double)eb.z;
    const double r = sqrt(r2), krf = (double)d.krf, crf = (double)d.crf;
    v = va + vb + qq * (1.0 / r + krf * r2 - crf);
    fs = fa + fb + qq * (1.0 / (r2 * r) - 2.0 * krf);
}

// F += F_sc(lam_to) - F_sc(lam_from) on each affected bead (8 lanes per bead)
template <typename R>
__global__ __launch_bounds__(WG) void k_scforce(Dev<R> d, Mv m, double lam_from, double lam_to,
                                                double delta, int defer)
{
    const int gid = blockIdx.x * WG + threadIdx.x;
    const int k0 = gid >> 3, s = gid & 7;
    const int na = min(*m.aff_n, m.aff_cap);
    const bool valid = k0 < na;
    const int i = valid ? m.aff_list[k0] : 0;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (valid) {
        const V4<R> pi = d.posq[i];
        const int ci = cls_of<R>(pi.w);
        const int mk = d.alch[i];
        const int ci2 = mk >= 0 ? (mk & 0xff) : ci;
        const int n1 = d.ncnt[i];
        // entries, owners and marks KB at a time per lane, as in k_dforce
        constexpr int KB = 4;
        for (int kb = s; kb < n1; kb += 8 * KB) {
            int ent[KB], own[KB], mrk[KB];
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                const int k = kb + 8 * b;
                ent[b] = k < n1 ? d.nbr[nbr_index(i, k, d.Kcap, d.lpb)] : 0;
            }
#pragma unroll
            for (int b = 0; b < KB; ++b)
                own[b] = kb + 8 * b < n1 ? owner_of(d.ghost_owner, d.N, ent[b] & JMASK) : 0;
#pragma unroll
            for (int b = 0; b < KB; ++b) mrk[b] = kb + 8 * b < n1 ? d.alch[own[b]] : -1;
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                if (kb + 8 * b >= n1) continue;
                const int en = ent[b], o = own[b], mj = mrk[b];
                const int j = en & JMASK, code = (int)((unsigned)en >> CODE_SHIFT);
                if (mk < 0 && mj < 0) continue;
                const V4<R> pj = d.posq[j];
                const int cj = cls_of<R>(d.posq[o].w);
                const int cj2 = mj >= 0 ? (mj & 0xff) : cj;
                const R xs = (code & 1) ? pi.x - d.L[0] : pi.x;
                const R ys = (code & 2) ? pi.y - d.L[1] : pi.y;
                const R zs = (code & 4) ? pi.z - d.L[2] : pi.z;
                const double dx = (double)xs - (double)pj.x, dy = (double)ys - (double)pj.y,
                             dz = (double)zs - (double)pj.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (!(r2 < d.rc2d)) continue;
                double v1, f1, v0, f0;
                sc_pair_d(d, ci, cj, ci2, cj2, r2, lam_to, delta, v1, f1);
                sc_pair_d(d, ci, cj, ci2, cj2, r2, lam_from, delta, v0, f0);
                const double fs = f1 - f0;
                fx += fs * dx; fy += fs * dy; fz += fs * dz;
            }
        }
    }
#pragma unroll
    for (int q = 4; q >= 1; q >>= 1) {
        fx += __shfl_xor(fx, q);
        fy += __shfl_xor(fy, q);
        fz += __shfl_xor(fz, q);
    }
    if (valid && s == 0) {
        if (defer) {   // applied by the segment boundary pass (k_sc_bridge)
            m.dsc[4 * (size_t)i] = fx; m.dsc[4 * (size_t)i + 1] = fy; m.dsc[4 * (size_t)i + 2] = fz;
        } else {
            V4<R> f = d.frc[i];
            f.x = (R)((double)f.x + fx); f.y = (R)((double)f.y + fy); f.z = (R)((double)f.z + fz);
            d.frc[i] = f;
        }
    }
}

// U_sc(lam1) - U_sc(lam0) over one changed bead's pairs (one wave per changed
// bead; pairs of two changed beads visited from both ends, weight 1/2)
template <typename R>
__global__ __launch_bounds__(64) void k_scdu(Dev<R> d, Mv m, double lam0, double lam1, double delta)
{
    const int e = blockIdx.x, lane = threadIdx.x;
    const int MC = m.maxcht;
    const int a = e / MC, q = e % MC;
    if (a >= m.r_n[0] || q >= m.r_nb[a]) {
        if (lane == 0) m.du_bead[e] = 0.0;
        return;
    }
    const int i = d.inv[m.r_bead[a * MC + q]];
    const V4<R> pi = d.posq[i];
    const int ci = cls_of<R>(pi.w);
    const int mk = d.alch[i];
    const int ci2 = mk & 0xff, tag = mk >> 8;
    const int n1 = d.ncnt[i];
    double du = 0.0;
    for (int k = lane; k < n1; k += 64) {
        const int en = d.nbr[nbr_index(i, k, d.Kcap, d.lpb)];
        const int j = en & JMASK, code = (int)((unsigned)en >> CODE_SHIFT);
        const V4<R> pj = d.posq[j];
        const int o = owner_of(d.ghost_owner, d.N, j);
        const int cj = cls_of<R>(d.posq[o].w);
        const int mj = d.alch[o];
        int cj2 = cj;
        double wgt = 1.0;
        if (mj >= 0 && (mj >> 8) == tag) { cj2 = mj & 0xff; wgt = 0.5; }
        const R xs = (code & 1) ? pi.x - d.L[0] : pi.x;
        const R ys = (code & 2) ? pi.y - d.L[1] : pi.y;
        const R zs = (code & 4) ? pi.z - d.L[2] : pi.z;
        const double dx = (double)xs - (double)pj.x, dy = (double)ys - (double)pj.y,
                     dz = (double)zs - (double)pj.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < d.rc2d) {
            double v1, f1, v0, f0;
            sc_pair_d(d, ci, cj, ci2, cj2, r2, lam1, delta, v1, f1);
            sc_pair_d(d, ci, cj, ci2, cj2, r2, lam0, delta, v0, f0);
            du += wgt * (v1 - v0);
        }
    }
    du = dwave_sum(du);
    if (lane == 0) m.du_bead[e] = du;
}

// F += dl (F_B - F_A) on the affected beads (a lambda increment, Eq. 2).
template <typename R>
__global__ void k_dlam(Dev<R> d, Mv m, R dl)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int na = min(*m.aff_n, m.aff_cap);
    if (k >= na) return;
    int i = m.aff_list[k];
    V4<R> f = d.frc[i], g = d.dfrc[i];
    f.x += dl * g.x; f.y += dl * g.y; f.z += dl * g.z;
    d.frc[i] = f;
}

// ------------------------------------------- topology-changing exchanges
// An exchange between kinds whose bonded terms differ changes the bonded
// energy and forces of both molecules.  In float64, from the stored
// coordinates, with the bonded partners' minimum-image separation taken as
// in the force pass (the coordinate beyond half a box shifted by L first).
__device__ __forceinline__ double sep_d(double xi, double xj, double L)
{
    double dx = xi - xj;
    if (dx > 0.5 * L) dx = (xi - L) - xj;
    else if (dx < -0.5 * L) dx = xi - (xj - L);
    return dx;
}

// Bonded energy of molecule mol as kind k at the current coordinates; with
// f, its forces are added to f[local bead][axis] times sgn.
template <typename R>
__device__ double mol_bonded(const Dev<R>& d, int mol, int k, double (*f)[3], double sgn)
{
    const int f0 = d.mol_first[mol];
    double u = 0.0;
    for (int q = 0; q < d.kb_n[k]; ++q) {
        const int bq = d.kb_off[k] + q;
        const int li = d.b_ij[2 * bq], lj = d.b_ij[2 * bq + 1];
        const V4<R> pi = d.posq[d.inv[f0 + li]], pj = d.posq[d.inv[f0 + lj]];
        const double dx = sep_d(pi.x, pj.x, d.Ld[0]), dy = sep_d(pi.y, pj.y, d.Ld[1]),
                     dz = sep_d(pi.z, pj.z, d.Ld[2]);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double kk = (double)d.b_par[2 * bq + 1], dr = r - (double)d.b_par[2 * bq];
        u += 0.5 * kk * dr * dr;
        if (f) {
            const double fs = -kk * dr / r * sgn;
            f[li][0] += fs * dx; f[li][1] += fs * dy; f[li][2] += fs * dz;
            f[lj][0] -= fs * dx; f[lj][1] -= fs * dy; f[lj][2] -= fs * dz;
        }
    }
    for (int q = 0; q < d.ka_n[k]; ++q) {
        const int aq = d.ka_off[k] + q;
        const int li = d.a_ijk[3 * aq], lj = d.a_ijk[3 * aq + 1], lk = d.a_ijk[3 * aq + 2];
        const V4<R> pi = d.posq[d.inv[f0 + li]], pj = d.posq[d.inv[f0 + lj]],
                    pk = d.posq[d.inv[f0 + lk]];
        const double u3[3] = { sep_d(pi.x, pj.x, d.Ld[0]), sep_d(pi.y, pj.y, d.Ld[1]),
                               sep_d(pi.z, pj.z, d.Ld[2]) };
        const double w3[3] = { sep_d(pk.x, pj.x, d.Ld[0]), sep_d(pk.y, pj.y, d.Ld[1]),
                               sep_d(pk.z, pj.z, d.Ld[2]) };
        const double uu = u3[0] * u3[0] + u3[1] * u3[1] + u3[2] * u3[2];
        const double ww = w3[0] * w3[0] + w3[1] * w3[1] + w3[2] * w3[2];
        const double nuw = sqrt(uu) * sqrt(ww);
        const double cth = (u3[0] * w3[0] + u3[1] * w3[1] + u3[2] * w3[2]) / nuw;
        const double kk = (double)d.a_par[2 * aq + 1], dc = cth - (double)d.a_par[2 * aq];
        u += 0.5 * kk * dc * dc;
        if (f) {
            const double pre = -kk * dc * sgn;
            for (int a = 0; a < 3; ++a) {
                const double dci = w3[a] / nuw - cth * u3[a] / uu;
                const double dck = u3[a] / nuw - cth * w3[a] / ww;
                f[li][a] += pre * dci;
                f[lk][a] += pre * dck;
                f[lj][a] -= pre * (dci + dck);
            }
        }
    }
    return u;
}

// du_bond[a] = scale (U_bonded(after) - U_bonded(before)) of trial a: X and
// Y in each other's kinds minus in their own (zero unless the kinds differ
// in their bonded terms).  One thread per trial.
template <typename R>
__global__ void k_bond_du(Dev<R> d, Mv m, double scale)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m.T) return;
    double du = 0.0;
    if (a < m.r_n[0]) {
        const int X = m.r_x[a], Y = m.r_y[a];
        const int kx = d.mol_kind[X], ky = d.mol_kind[Y];
        if (d.ktopo[kx * d.nk + ky])
            du = scale * ((mol_bonded(d, X, ky, nullptr, 0.0) + mol_bonded(d, Y, kx, nullptr, 0.0)) -
                          (mol_bonded(d, X, kx, nullptr, 0.0) + mol_bonded(d, Y, ky, nullptr, 0.0)));
    }
    m.du_bond[a] = du;
}

// F_new - F_old of the bonded terms on the beads of each side of a trial
// (thread 2 a + side: X, Y), kept in dfb and added to the stored forces
// times scale; with only_accepted, trials that were not accepted are left
// alone.  Zero unless the kinds differ in their bonded terms.
template <typename R>
__global__ void k_bond_dforce(Dev<R> d, Mv m, double scale, int only_accepted)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = e >> 1, side = e & 1;
    if (a >= m.r_n[0]) return;
    if (only_accepted && !m.r_acc[a]) return;
    const int X = m.r_x[a], Y = m.r_y[a];
    const int mol = side ? Y : X, other = side ? X : Y;
    const int kold = d.mol_kind[mol], knew = d.mol_kind[other];
    double f[MAXKN_TOPO][3];
    for (int l = 0; l < MAXKN_TOPO; ++l) f[l][0] = f[l][1] = f[l][2] = 0.0;
    const bool topo = d.ktopo[kold * d.nk + knew] != 0;
    if (topo) {
        mol_bonded(d, mol, knew, f, 1.0);
        mol_bonded(d, mol, kold, f, -1.0);
    }
    double* out = m.dfb + (size_t)e * MAXKN_TOPO * 3;
    const int f0 = d.mol_first[mol], n = d.kn[kold];
    for (int l = 0; l < MAXKN_TOPO; ++l) {
        out[3 * l] = f[l][0]; out[3 * l + 1] = f[l][1]; out[3 * l + 2] = f[l][2];
        if (topo && l < n && scale != 0.0) {
            const int sl = d.inv[f0 + l];
            V4<R> g = d.frc[sl];
            g.x = (R)((double)g.x + scale * f[l][0]);
            g.y = (R)((double)g.y + scale * f[l][1]);
            g.z = (R)((double)g.z + scale * f[l][2]);
            d.frc[sl] = g;
        }
    }
}

// F += dl (F_B - F_A) of the bonded terms (an MDAS lambda increment).
template <typename R>
__global__ void k_bond_dlam(Dev<R> d, Mv m, double dl)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = e >> 1, side = e & 1;
    if (a >= m.r_n[0]) return;
    const int mol = side ? m.r_y[a] : m.r_x[a];
    const int f0 = d.mol_first[mol], n = min(d.kn[d.mol_kind[mol]], MAXKN_TOPO);
    const double* in = m.dfb + (size_t)e * MAXKN_TOPO * 3;
    for (int l = 0; l < n; ++l) {
        const int sl = d.inv[f0 + l];
        V4<R> g = d.frc[sl];
        g.x = (R)((double)g.x + dl * in[3 * l]);
        g.y = (R)((double)g.y + dl * in[3 * l + 1]);
        g.z = (R)((double)g.z + dl * in[3 * l + 2]);
        d.frc[sl] = g;
    }
}

// After accepted exchanges between kinds with different bonded terms: the
// molecules' bonded records (bead-id order) and their slot-ordered copies
// rewritten from their new kinds' templates (run after the commit).
template <typename R>
__global__ void k_bt_refresh(Dev<R> d, Mv m, int mode)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = e >> 1, side = e & 1;
    if (a >= m.r_n[0]) return;
    const bool acc = mode == 0 ? (m.r_acc[a] != 0) : (m.md[2] != 0.0);
    if (!acc) return;
    const int X = m.r_x[a], Y = m.r_y[a];
    const int mol = side ? Y : X;
    const int k = d.mol_kind[mol], ko = d.mol_kind[side ? X : Y];
    if (!d.ktopo[k * d.nk + ko]) return;
    const int f0 = d.mol_first[mol];
    for (int l = 0; l < d.kn[k]; ++l) {
        const int b = f0 + l, sl = d.inv[b];
        for (int t = 0; t < MAXBT; ++t) {
            const int4 tp = d.ktpl[(size_t)(d.kbead_off[k] + l) * MAXBT + t];
            const bool on = tp.x >= 0;
            const int p1 = on ? f0 + tp.y : b, p2 = on && tp.z >= 0 ? f0 + tp.z : -1;
            d.bt[(size_t)b * MAXBT + t] = make_int4(on ? tp.x : -1, p1, p2, on ? tp.w : 0);
            d.bslot[(size_t)sl * MAXBT + t] =
                make_int4(on ? tp.x : -1, d.inv[p1], p2 >= 0 ? d.inv[p2] : sl, on ? tp.w : 0);
        }
    }
}

// Apply accepted exchanges: new classes and molecule kinds.
template <typename R>
__global__ void k_commit(Dev<R> d, Mv m, int mode)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int MC = m.maxcht;
    int a = e / MC, q = e % MC;
    if (a >= m.r_n[0]) return;
    bool acc = mode == 0 ? (m.r_acc[a] != 0) : (m.md[2] != 0.0);
    if (q == 0 && acc) {
        int X = m.r_x[a], Y = m.r_y[a];
        int kx = d.mol_kind[X];
        d.mol_kind[X] = d.mol_kind[Y];
        d.mol_kind[Y] = kx;
    }
    if (q >= m.r_nb[a]) return;
    int s = d.inv[m.r_bead[a * MC + q]];
    if (acc) {
        V4<R> p = d.posq[s];
        p.w = cls_to<R>(m.r_cls[a * MC + q]);
        d.posq[s] = p;
        // the bead's periodic images take the new class too (their record:
        // entries g | code << CODE_SHIFT, -1 unused, the second half read only
        // when the first is full)
        const int4* gl = reinterpret_cast<const int4*>(d.glist) + 2 * s;
        const int4 g0 = gl[0];
        int ge[8] = { g0.x, g0.y, g0.z, g0.w, -1, -1, -1, -1 };
        if (g0.w != -1) {
            const int4 g1 = gl[1];
            ge[4] = g1.x; ge[5] = g1.y; ge[6] = g1.z; ge[7] = g1.w;
        }
        for (int k = 0; k < 8 && ge[k] != -1; ++k) {
            const int g = d.N + (ge[k] & JMASK);
            V4<R> pg = d.posq[g];
            pg.w = p.w;
            d.posq[g] = pg;
        }
    }
    d.alch[s] = -1;
}

// MDAS: w += dl dU ; accept test u < exp(-w/kT) (Eq. 3)
__global__ void k_work(double* md, double dl) { md[0] += dl * md[1]; }

template <typename R>
__global__ void k_mdas_accept(Dev<R> d, Mv m)
{
    uint4 w = draw(d.seed, 0u, d.ctr[CT_CYCLE], ST_MDAS_ACCEPT);
    double u = u53(w.x, w.y);
    m.md[3] = u;
    const bool acc = u < exp(-m.md[0] / d.kTd);
    m.md[2] = acc ? 1.0 : 0.0;
    if (acc) d.ctr[CT_MDAS_ACC] += 1;
}

// Snapshot / restore of the per-slot state around an alchemical trajectory.
template <typename R>
__global__ void k_snapshot(Dev<R> d, Mv m, int restore)
{
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    V4<R>* sp = (V4<R>*)m.snap_posq;
    V4<R>* sv = (V4<R>*)m.snap_vel;
    V4<R>* sf = (V4<R>*)m.snap_frc;
    if (!restore) {
        sp[i] = d.posq[i]; sv[i] = d.vel[i]; sf[i] = d.frc[i]; m.snap_orig[i] = d.orig[i];
    } else {
        if (m.md[2] != 0.0) return;   // accepted: keep the lambda = 1 state
        d.posq[i] = sp[i]; d.vel[i] = sv[i]; d.frc[i] = sf[i]; d.orig[i] = m.snap_orig[i];
        d.alch[i] = -1;
    }
}

// Per-kind prefix counts over the kind's family member list.
// Prefix counts of `kind` over the member list mem[n] (out[k]: members of
// that kind before position k, out[n] the total) and the members of other
// kinds in ascending order (oth); all 1024 threads of the block call it.
template <typename R>
__device__ void kcnt_list(const Dev<R>& d, const int* __restrict__ mem, int nf, int kind, int* out,
                          int* oth)
{
    __shared__ int part[1024];
    // a thread's segment (up to KU molecules) in chunks of KC loads in flight
    constexpr int KU = 48, KC = 16;
    const int t = threadIdx.x;
    const int per = (nf + 1023) / 1024;
    const int b = t * per, e = min(nf, b + per);
    int s = 0;
    unsigned long long same = 0;
    if (per <= KU) {
#pragma unroll
        for (int c0 = 0; c0 < KU; c0 += KC) {
            if (b + c0 >= e) break;
            int mk[KC];
#pragma unroll
            for (int u = 0; u < KC; ++u) mk[u] = b + c0 + u < e ? mem[b + c0 + u] : -1;
#pragma unroll
            for (int u = 0; u < KC; ++u)
                if (mk[u] >= 0 && d.mol_kind[mk[u]] == kind) same |= 1ull << (c0 + u);
        }
        s = __popcll(same);
    } else {
        for (int k = b; k < e; ++k) s += d.mol_kind[mem[k]] == kind;
    }
    __syncthreads();   // part may still be read by a previous call
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    if (per <= KU) {
#pragma unroll
        for (int c0 = 0; c0 < KU; c0 += KC) {
            if (b + c0 >= e) break;
            int mk[KC];
#pragma unroll
            for (int u = 0; u < KC; ++u) mk[u] = b + c0 + u < e ? mem[b + c0 + u] : -1;
#pragma unroll
            for (int u = 0; u < KC; ++u) {
                if (b + c0 + u < e) {
                    const bool sm = (same >> (c0 + u)) & 1ull;
                    out[b + c0 + u] = run;
                    if (!sm) oth[b + c0 + u - run] = mk[u];   // members of other kinds, ascending
                    run += sm ? 1 : 0;
                }
            }
        }
    } else {
        for (int k = b; k < e; ++k) {
            const int mm = mem[k];
            const bool sm = d.mol_kind[mm] == kind;
            out[k] = run;
            if (!sm) oth[k - run] = mm;
            run += sm;
        }
    }
    if (t == 1023) out[nf] = part[1023];
}

// Kind counts of one kind over its family, and (within-region exchanges)
// over each region of the family.
template <typename R>
__global__ __launch_bounds__(1024) void k_kcnt(Dev<R> d, Mv m, int kind0, int batch_done)
{
    // batch_done: this launch closes an exchange batch, whose counter it advances
    if (batch_done && blockIdx.x == 0 && threadIdx.x == 0) d.ctr[CT_BATCH] += 1;
    const int kind = kind0 + blockIdx.x;   // one work-group per kind
    const int f = m.fam_of_kind[kind];
    if (f < 0) return;
    const int f0 = m.fam_off[f], nf = m.fam_off[f + 1] - f0;
    kcnt_list(d, m.fam_mem + f0, nf, kind, m.kcnt + kind * m.fam_stride,
              m.others + kind * m.fam_stride);
    if (m.xmode == 1)
        for (int r = 0; r < 2; ++r) {
            const int o0 = m.reg_off[2 * f + r], nr = m.reg_off[2 * f + r + 1] - o0;
            const int base = (kind * 2 + r) * m.fam_stride;
            kcnt_list(d, m.reg_mem + o0, nr, kind, m.kcnt_r + base, m.others_r + base);
        }
}

// ----------------------------------------------------------------- launch
// Chunk sizes: SEL_C0, 4 SEL_C0, then SEL_CMAX, until they cover the draw
// cap; one more of SEL_CMAX in reserve (a chunk ends early only where a
// candidate has more than SEL_CAPC earlier conflicts or the chunk's lists
// outgrow SEL_LDS), then the one-draw-at-a-time tail.  The chunking does
// not change the admitted trials, only how many rounds find them.  A small
// first chunk pays: the later chunks' draws are filtered against the trials
// admitted before, and most of them fall out there.  Measured on the
// 95,876-bead bilayer, 256 trials plus 2 MD steps per batch: 0.530 ms with
// chunks of 1k, 1k, 2k, 4k, 8k; 0.515 ms with 2k, 8k, ...; 0.502 ms with
// 1k, 8k, ...; 0.490 ms with 1k, 2k, 8k, ...; 0.485 ms with this sequence.
// (A first chunk of 8192 draws alone took 350 us to resolve.)
template <typename R>
void launch_select(const Dev<R>& d, const Mv& m, int n_want, int draw_cap, int mode,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, st, m, n_want);
    long long covered = 0;
    int reserve = 1, ck = SEL_C0, k = 0;
    while (true) {
        if (covered >= draw_cap) {
            if (reserve == 0) break;
            --reserve;
            ck = SEL_CMAX;
        }
        hipLaunchKernelGGL(k_sel_draw<R>, dim3(ck / 4), dim3(256), 0, st, d, m, draw_cap, mode, ck);
        hipLaunchKernelGGL(k_sel_conf<R>, dim3(ck / 4), dim3(256), 0, st, d, m, mode, ck);
        hipLaunchKernelGGL(k_sel_resolve<R>, dim3(1), dim3(1024), 0, st, d, m, n_want, draw_cap,
                           mode, ck);
        covered += ck;
        ck = ++k == 1 ? 4 * SEL_C0 : SEL_CMAX;
    }
    hipLaunchKernelGGL(k_sel_tail<R>, dim3(1), dim3(64), 0, st, d, m, n_want, draw_cap, mode);
}

template <typename R>
void launch_mark(const Dev<R>& d, const Mv& m, int mode, int T, hipStream_t st)
{
    int n = T * m.maxcht;
    hipLaunchKernelGGL(k_mark<R>, dim3((n + 255) / 256), dim3(256), 0, st, d, m, mode);
}


template <typename R>
void launch_du(const Dev<R>& d, const Mv& m, int T, hipStream_t st)
{
    hipLaunchKernelGGL(k_du_bead<R>, dim3(T * m.maxcht), dim3(64), 0, st, d, m);
}

template <typename R>
void launch_trial_accept(const Dev<R>& d, const Mv& m, int T, hipStream_t st)
{
    hipLaunchKernelGGL(k_trial_accept<R>, dim3((T + 255) / 256), dim3(256), 0, st, d, m);
}

template <typename R>
void launch_du_total(const Dev<R>& d, const Mv& m, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_du_total<R>, dim3(1), dim3(64), 0, st, d, m, out);
}

template <typename R>
void launch_aff_build(const Dev<R>& d, const Mv& m, int only_accepted, int T, bool zero,
                      hipStream_t st)
{
    // zero = false: k_mark of the same trials has emptied the set
    if (zero) hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, m.aff_n);
    hipLaunchKernelGGL(k_aff_mark<R>, dim3(T * m.maxcht), dim3(64), 0, st, d, m, only_accepted);
}

template <typename R>
void launch_aff_clear(const Dev<R>& d, const Mv& m, hipStream_t st)
{
    hipLaunchKernelGGL(k_aff_clear<R>, dim3((m.aff_cap + 255) / 256), dim3(256), 0, st, d, m);
}

template <typename R>
void launch_dforce(const Dev<R>& d, const Mv& m, R scale, hipStream_t st)
{
    int n = m.aff_cap * 8;
    hipLaunchKernelGGL(k_dforce<R>, dim3((n + WG - 1) / WG), dim3(WG), 0, st, d, m, scale);
}

template <typename R>
void launch_scforce(const Dev<R>& d, const Mv& m, double lam_from, double lam_to, double delta,
                    hipStream_t st, bool defer)
{
    int n = m.aff_cap * 8;
    hipLaunchKernelGGL(k_scforce<R>, dim3((n + WG - 1) / WG), dim3(WG), 0, st, d, m, lam_from, lam_to,
                       delta, defer ? 1 : 0);
}

template <typename R>
void launch_scdu(const Dev<R>& d, const Mv& m, int T, double lam0, double lam1, double delta,
                 hipStream_t st)
{
    hipLaunchKernelGGL(k_scdu<R>, dim3(T * m.maxcht), dim3(64), 0, st, d, m, lam0, lam1, delta);
}

template <typename R>
void launch_dlam(const Dev<R>& d, const Mv& m, R dl, hipStream_t st)
{
    hipLaunchKernelGGL(k_dlam<R>, dim3((m.aff_cap + 255) / 256), dim3(256), 0, st, d, m, dl);
}

template <typename R>
void launch_bond_du(const Dev<R>& d, const Mv& m, double scale, hipStream_t st)
{
    hipLaunchKernelGGL(k_bond_du<R>, dim3((m.T + 255) / 256), dim3(256), 0, st, d, m, scale);
}

template <typename R>
void launch_bond_dforce(const Dev<R>& d, const Mv& m, double scale, int only_accepted, hipStream_t st)
{
    hipLaunchKernelGGL(k_bond_dforce<R>, dim3((2 * m.T + 63) / 64), dim3(64), 0, st, d, m, scale,
                       only_accepted);
}

template <typename R>
void launch_bond_dlam(const Dev<R>& d, const Mv& m, double dl, hipStream_t st)
{
    hipLaunchKernelGGL(k_bond_dlam<R>, dim3((2 * m.T + 63) / 64), dim3(64), 0, st, d, m, dl);
}

template <typename R>
void launch_bt_refresh(const Dev<R>& d, const Mv& m, int mode, hipStream_t st)
{
    hipLaunchKernelGGL(k_bt_refresh<R>, dim3((2 * m.T + 63) / 64), dim3(64), 0, st, d, m, mode);
}

template <typename R>
void launch_commit(const Dev<R>& d, const Mv& m, int mode, int T, hipStream_t st)
{
    int n = T * m.maxcht;
    hipLaunchKernelGGL(k_commit<R>, dim3((n + 255) / 256), dim3(256), 0, st, d, m, mode);
}

void launch_work(double* md, double dl, hipStream_t st)
{
    hipLaunchKernelGGL(k_work, dim3(1), dim3(1), 0, st, md, dl);
}

template <typename R>
void launch_mdas_accept(const Dev<R>& d, const Mv& m, hipStream_t st)
{
    hipLaunchKernelGGL(k_mdas_accept<R>, dim3(1), dim3(1), 0, st, d, m);
}

template <typename R>
void launch_snapshot(const Dev<R>& d, const Mv& m, int restore, hipStream_t st)
{
    hipLaunchKernelGGL(k_snapshot<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, m, restore);
}

template <typename R>
void launch_kcnt(const Dev<R>& d, const Mv& m, int kind0, int nkinds, int batch_done, hipStream_t st)
{
    if (nkinds <= 0) return;
    hipLaunchKernelGGL(k_kcnt<R>, dim3(nkinds), dim3(1024), 0, st, d, m, kind0, batch_done);
}

#define INSTM(R)                                                                         \
    template void launch_select<R>(const Dev<R>&, const Mv&, int, int, int, hipStream_t); \
    template void launch_mark<R>(const Dev<R>&, const Mv&, int, int, hipStream_t);        \
    template void launch_du<R>(const Dev<R>&, const Mv&, int, hipStream_t);               \
    template void launch_trial_accept<R>(const Dev<R>&, const Mv&, int, hipStream_t);     \
    template void launch_du_total<R>(const Dev<R>&, const Mv&, double*, hipStream_t);     \
    template void launch_aff_build<R>(const Dev<R>&, const Mv&, int, int, bool, hipStream_t); \
    template void launch_aff_clear<R>(const Dev<R>&, const Mv&, hipStream_t);             \
    template void launch_dforce<R>(const Dev<R>&, const Mv&, R, hipStream_t);             \
    template void launch_dlam<R>(const Dev<R>&, const Mv&, R, hipStream_t);               \
    template void launch_scforce<R>(const Dev<R>&, const Mv&, double, double, double,      \
                                    hipStream_t, bool);                                   \
    template void launch_scdu<R>(const Dev<R>&, const Mv&, int, double, double, double,    \
                                 hipStream_t);                                            \
    template void launch_commit<R>(const Dev<R>&, const Mv&, int, int, hipStream_t);      \
    template void launch_bond_du<R>(const Dev<R>&, const Mv&, double, hipStream_t);       \
    template void launch_bond_dforce<R>(const Dev<R>&, const Mv&, double, int, hipStream_t); \
    template void launch_bond_dlam<R>(const Dev<R>&, const Mv&, double, hipStream_t);     \
    template void launch_bt_refresh<R>(const Dev<R>&, const Mv&, int, hipStream_t);       \
    template void launch_mdas_accept<R>(const Dev<R>&, const Mv&, hipStream_t);           \
    template void launch_snapshot<R>(const Dev<R>&, const Mv&, int, hipStream_t);         \
    template void launch_kcnt<R>(const Dev<R>&, const Mv&, int, int, int, hipStream_t);
INSTM(float)
INSTM(double)

}  // namespace mbx
