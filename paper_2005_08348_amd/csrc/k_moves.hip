// k_moves.hip -- exchange moves of the paper's Theory section on the GPU.
//
// MC-MD (Eq. 1): a batch of exchange trials is drawn in counter order and
// filtered greedily (a candidate is admitted when it shares no molecule with,
// and none of its changed beads is within r_cut of a changed bead of, an
// earlier admitted candidate).  The filter is sequential by definition; here
// one work-group examines CHUNK candidates at a time: all candidates are
// drawn and located in parallel, conflicts between them are found through a
// spatial hash, and the lexicographically-first admission is resolved by
// parallel rounds (a candidate is in once every earlier conflicting
// candidate is out, out as soon as one is in), which reproduces the
// sequential order exactly.  Each admitted trial's dU = U(after) - U(before)
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

// push entry e into the list of `cell` for epoch ep (64-bit head: epoch|index)
__device__ __forceinline__ void hash_push(unsigned long long* head, int* next, int cell, int e,
                                          unsigned ep)
{
    unsigned long long nw = ((unsigned long long)ep << 32) | (unsigned)e;
    unsigned long long old = head[cell];
    while (true) {
        int nxt = ((unsigned)(old >> 32) == ep) ? (int)(unsigned)(old & 0xffffffffu) : -1;
        next[e] = nxt;
        unsigned long long got = atomicCAS(&head[cell], old, nw);
        if (got == old) break;
        old = got;
    }
}

__device__ __forceinline__ int hash_first(const unsigned long long* head, int cell, unsigned ep)
{
    unsigned long long h = head[cell];
    return ((unsigned)(h >> 32) == ep) ? (int)(unsigned)(h & 0xffffffffu) : -1;
}

__device__ __forceinline__ void conf_add(int* lst, int& n, int t2, bool& ovf)
{
    for (int q = 0; q < n && q < MAXCONF; ++q)
        if (lst[q] == t2) return;
    if (n < MAXCONF) lst[n] = t2; else ovf = true;
    ++n;
}

// Candidate selection.  mode 0: exchange batch (stream 1, counter = batch,
// spatial filter); mode 1: MDAS pairs (stream 3, counter = cycle, distinct
// molecules only).  One work-group of CHUNK threads.
template <typename R>
__global__ __launch_bounds__(CHUNK) void k_select(Dev<R> d, Mv m, int n_want, int draw_cap,
                                                  int mode)
{
    __shared__ int st[CHUNK];          // 0 undecided, 1 in, 2 out
    __shared__ int ord[CHUNK];
    __shared__ int s_adm, s_d0, s_chg, s_nin, s_stop;
    const int t = threadIdx.x;
    const int T = n_want;
    const long long ctrv = d.ctr[mode == 0 ? CT_BATCH : CT_CYCLE];
    const unsigned stream = mode == 0 ? ST_SWAP_DRAW : ST_MDAS_SELECT;
    const unsigned base = (unsigned)m.r_n[2];
    const unsigned callstamp = base + 1u;
    unsigned long long* hhead = (unsigned long long*)m.h_head;
    unsigned long long* mhead = (unsigned long long*)m.m_head;
    const int MC = m.maxcht;
    if (t == 0) { s_adm = 0; s_d0 = 0; s_stop = 0; }
    __syncthreads();
    int chunk = 0;
    while (true) {
        if (s_stop || s_adm >= T || s_d0 >= draw_cap) break;
        const unsigned ep = base + 2u + (unsigned)chunk;
        const int base_d = s_d0;
        // ---- phase A: draw and locate candidate d0 + t
        const int dd = base_d + t;
        int flag = 1, X = -1, Y = -1, nb = 0;
        if (dd < draw_cap && m.n_sw > 0) {
            uint4 w = draw(d.seed, (uint32_t)dd, ctrv, stream);
            X = m.sw_list[pick(w.x, (uint32_t)m.n_sw)];
            int kx = d.mol_kind[X];
            int f = m.fam_of_kind[kx];
            int f0 = m.fam_off[f], nf = m.fam_off[f + 1] - f0;
            const int* kc = m.kcnt + kx * m.fam_stride;
            int noth = nf - kc[nf];
            if (noth > 0) {
                uint32_t k = pick(w.y, (uint32_t)noth);
                // smallest p with (p + 1) - kc[p + 1] > k
                int lo = 0, hi = nf - 1;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if ((mid + 1) - kc[mid + 1] > (int)k) hi = mid; else lo = mid + 1;
                }
                Y = m.fam_mem[f0 + lo];
                int ky = d.mol_kind[Y];
                flag = 0;
                if (m.used[X] == (int)callstamp || m.used[Y] == (int)callstamp) flag = 2;
                int nch = m.chg_n[kx * d.nk + ky];
                const int* loc = m.chg_loc + (kx * d.nk + ky) * MAXCH;
                for (int q = 0; q < nch; ++q) {
                    int l = loc[q];
                    int bx = d.mol_first[X] + l, by = d.mol_first[Y] + l;
                    m.c_bead[t * MC + q] = bx;
                    m.c_cls[t * MC + q] = d.kcls[d.kbead_off[ky] + l];
                    m.c_bead[t * MC + nch + q] = by;
                    m.c_cls[t * MC + nch + q] = d.kcls[d.kbead_off[kx] + l];
                }
                nb = 2 * nch;
                for (int q = 0; q < nb; ++q) {
                    V4<R> p = d.posq[d.inv[m.c_bead[t * MC + q]]];
                    double* cp = m.c_pos + 3 * (t * MC + q);
                    cp[0] = (double)p.x; cp[1] = (double)p.y; cp[2] = (double)p.z;
                }
            }
        }
        m.c_x[t] = X; m.c_y[t] = Y; m.c_nb[t] = nb; m.c_flag[t] = flag;
        __syncthreads();
        // ---- phase B: hash this chunk's changed beads and molecules, plus
        // the changed beads of the trials admitted so far
        if (mode == 0) {
            if (flag != 1)
                for (int q = 0; q < nb; ++q) {
                    int c[3];
                    int cell = hash_cell(d, m, m.c_pos + 3 * (t * MC + q), c);
                    int e = t * MC + q;
                    m.h_owner[e] = t;
                    hash_push(hhead, m.h_next, cell, e, ep);
                }
            for (int a = t; a < s_adm; a += CHUNK) {
                for (int q = 0; q < m.r_nb[a]; ++q) {
                    int e = CHUNK * MC + a * MC + q;
                    double* hp = m.h_pos + 3 * e;
                    V4<R> p = d.posq[d.inv[m.r_bead[a * MC + q]]];
                    hp[0] = (double)p.x; hp[1] = (double)p.y; hp[2] = (double)p.z;
                    int c[3];
                    int cell = hash_cell(d, m, hp, c);
                    m.h_owner[e] = -1 - a;
                    hash_push(hhead, m.h_next, cell, e, ep);
                }
            }
        }
        if (flag != 1) {
            hash_push(mhead, m.m_next, X % m.mh, 2 * t, ep);
            m.m_owner[2 * t] = t;
            hash_push(mhead, m.m_next, Y % m.mh, 2 * t + 1, ep);
            m.m_owner[2 * t + 1] = t;
        }
        __syncthreads();
        // ---- phase C: conflicts
        int ncf = 0;
        bool ovf = false;
        int* cl = m.c_conf + t * MAXCONF;
        if (flag == 0) {
            // shared molecules with earlier candidates of this chunk
            for (int w2 = 0; w2 < 2; ++w2) {
                int mol = w2 ? Y : X;
                for (int e = hash_first(mhead, mol % m.mh, ep); e >= 0; e = m.m_next[e]) {
                    int o = m.m_owner[e];
                    if (o >= t) continue;
                    int om = (e & 1) ? m.c_y[o] : m.c_x[o];
                    if (om == mol) conf_add(cl, ncf, o, ovf);
                }
            }
            if (mode == 0) {
                for (int q = 0; q < nb && flag == 0; ++q) {
                    const double* pq = m.c_pos + 3 * (t * MC + q);
                    int c[3];
                    hash_cell(d, m, pq, c);
                    for (int o27 = 0; o27 < 27 && flag == 0; ++o27) {
                        int cx = (c[0] + o27 / 9 - 1 + m.hnc[0]) % m.hnc[0];
                        int cy = (c[1] + (o27 / 3) % 3 - 1 + m.hnc[1]) % m.hnc[1];
                        int cz = (c[2] + o27 % 3 - 1 + m.hnc[2]) % m.hnc[2];
                        int cell = (cx * m.hnc[1] + cy) * m.hnc[2] + cz;
                        for (int e = hash_first(hhead, cell, ep); e >= 0; e = m.h_next[e]) {
                            int o = m.h_owner[e];
                            if (o >= t) continue;   // later candidates and self
                            const double* pe = (o < 0) ? m.h_pos + 3 * e : m.c_pos + 3 * e;
                            if (mi_dist2(d, pq, pe) < d.rc2d) {
                                if (o < 0) flag = 2;
                                else conf_add(cl, ncf, o, ovf);
                            }
                        }
                    }
                }
            }
        }
        m.c_conf_n[t] = ovf ? -1 : ncf;
        st[t] = (flag != 0) ? 2 : 0;
        __syncthreads();
        // ---- phase D: resolve the lexicographically-first admission
        while (true) {
            if (t == 0) s_chg = 0;
            __syncthreads();
            int nst = st[t];
            if (nst == 0) {
                int cn = m.c_conf_n[t];
                if (cn >= 0) {
                    bool anyin = false, anyund = false;
                    for (int q = 0; q < cn; ++q) {
                        int s2 = st[cl[q]];
                        anyin |= (s2 == 1);
                        anyund |= (s2 == 0);
                    }
                    nst = anyin ? 2 : (anyund ? 0 : 1);
                } else {
                    // too many conflicts to list: compare with every earlier candidate
                    bool anyin = false, anyund = false;
                    for (int o = 0; o < t; ++o) {
                        int s2 = st[o];
                        if (s2 == 2) continue;
                        bool cf = (m.c_x[o] == X || m.c_x[o] == Y || m.c_y[o] == X || m.c_y[o] == Y);
                        if (mode == 0)
                            for (int q = 0; q < nb && !cf; ++q)
                                for (int q2 = 0; q2 < m.c_nb[o] && !cf; ++q2)
                                    cf = mi_dist2(d, m.c_pos + 3 * (t * MC + q),
                                                  m.c_pos + 3 * (o * MC + q2)) < d.rc2d;
                        if (!cf) continue;
                        anyin |= (s2 == 1);
                        anyund |= (s2 == 0);
                    }
                    nst = anyin ? 2 : (anyund ? 0 : 1);
                }
            }
            __syncthreads();
            if (nst != st[t]) { st[t] = nst; s_chg = 1; }
            __syncthreads();
            if (!s_chg) break;
        }
        // ---- phase E: take admitted candidates in draw order
        if (t == 0) {
            int need = T - s_adm, k = 0, last = -1;
            for (int q = 0; q < CHUNK && k < need; ++q)
                if (st[q] == 1) { ord[k++] = q; last = q; }
            s_nin = k;
            if (k == need && last >= 0) { s_d0 = base_d + last + 1; s_stop = 1; }
            else s_d0 = base_d + CHUNK;
        }
        __syncthreads();
        if (t < s_nin) {
            int q = ord[t], a = s_adm + t;
            m.r_draw[a] = base_d + q;
            m.r_x[a] = m.c_x[q];
            m.r_y[a] = m.c_y[q];
            m.r_nb[a] = m.c_nb[q];
            for (int e = 0; e < m.c_nb[q]; ++e) {
                m.r_bead[a * MC + e] = m.c_bead[q * MC + e];
                m.r_cls[a * MC + e] = m.c_cls[q * MC + e];
            }
            m.used[m.c_x[q]] = (int)callstamp;
            m.used[m.c_y[q]] = (int)callstamp;
        }
        __syncthreads();
        if (t == 0) s_adm += s_nin;
        ++chunk;
        __syncthreads();
    }
    if (t == 0) {
        m.r_n[0] = s_adm;
        m.r_n[1] = s_d0 < draw_cap ? s_d0 : draw_cap;
        m.r_n[2] = (int)(base + 2u + (unsigned)chunk);
    }
}

// Mark the changed beads of the admitted trials (tag = trial for exchange
// batches, 0 for MDAS) with their new class.
template <typename R>
__global__ void k_mark(Dev<R> d, Mv m, int mode)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int MC = m.maxcht;
    int a = e / MC, q = e % MC;
    if (a >= m.r_n[0] || q >= m.r_nb[a]) return;
    int s = d.inv[m.r_bead[a * MC + q]];
    d.alch[s] = m.r_cls[a * MC + q] | ((mode == 0 ? a : 0) << 8);
}

// Clear the marks (all admitted trials, or only the rejected ones).
template <typename R>
__global__ void k_unmark(Dev<R> d, Mv m, int only_rejected)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int MC = m.maxcht;
    int a = e / MC, q = e % MC;
    if (a >= m.r_n[0] || q >= m.r_nb[a]) return;
    if (only_rejected && m.r_acc[a]) return;
    d.alch[d.inv[m.r_bead[a * MC + q]]] = -1;
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
    const int n0 = d.nseg0[i], n1 = d.ncnt[i];
    double du = 0.0;
    for (int k = lane; k < n1; k += 64) {
        int en = d.nbr[nbr_index(i, k, d.Kcap, d.lpb)];
        int j = en & JMASK, code = (int)((unsigned)en >> CODE_SHIFT);
        if (k < n0) code = 0;
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
    uint4 w = draw(d.seed, (uint32_t)m.r_draw[a], d.ctr[CT_BATCH], ST_SWAP_ACCEPT);
    double u = u53(w.x, w.y);
    int acc = u < exp(-du / d.kTd);
    m.r_du[a] = du;
    m.r_u[a] = u;
    m.r_acc[a] = acc;
}

// Total dU over every admitted change (MDAS: U_B - U_A at the current x).
template <typename R>
__global__ void k_du_total(Dev<R> d, Mv m, double* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int MC = m.maxcht;
    double s = 0.0;
    for (int a = 0; a < m.r_n[0]; ++a)
        for (int q = 0; q < m.r_nb[a]; ++q) s += m.du_bead[a * MC + q];
    *out = s;
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
        const int n0 = d.nseg0[i], n1 = d.ncnt[i];
        for (int k = s; k < n1; k += 8) {
            int en = d.nbr[nbr_index(i, k, d.Kcap, d.lpb)];
            int j = en & JMASK, code = (int)((unsigned)en >> CODE_SHIFT);
            if (k < n0) code = 0;
            int o = owner_of(d.ghost_owner, d.N, j);
            int mj = d.alch[o];
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
    m.md[2] = (u < exp(-m.md[0] / d.kTd)) ? 1.0 : 0.0;
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
template <typename R>
__global__ void k_kcnt(Dev<R> d, Mv m, int kind)
{
    __shared__ int part[1024];
    int f = m.fam_of_kind[kind];
    if (f < 0) return;
    int f0 = m.fam_off[f], nf = m.fam_off[f + 1] - f0;
    int* out = m.kcnt + kind * m.fam_stride;
    int t = threadIdx.x;
    int per = (nf + 1023) / 1024;
    int b = t * per, e = min(nf, b + per);
    int s = 0;
    for (int k = b; k < e; ++k) s += d.mol_kind[m.fam_mem[f0 + k]] == kind;
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int k = b; k < e; ++k) { out[k] = run; run += d.mol_kind[m.fam_mem[f0 + k]] == kind; }
    if (t == 1023) out[nf] = part[1023];
}

// ----------------------------------------------------------------- launch
template <typename R>
void launch_select(const Dev<R>& d, const Mv& m, int n_want, int draw_cap, int mode,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_select<R>, dim3(1), dim3(CHUNK), 0, st, d, m, n_want, draw_cap, mode);
}

template <typename R>
void launch_mark(const Dev<R>& d, const Mv& m, int mode, int T, hipStream_t st)
{
    int n = T * m.maxcht;
    hipLaunchKernelGGL(k_mark<R>, dim3((n + 255) / 256), dim3(256), 0, st, d, m, mode);
}

template <typename R>
void launch_unmark(const Dev<R>& d, const Mv& m, int only_rejected, int T, hipStream_t st)
{
    int n = T * m.maxcht;
    hipLaunchKernelGGL(k_unmark<R>, dim3((n + 255) / 256), dim3(256), 0, st, d, m, only_rejected);
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
void launch_aff_build(const Dev<R>& d, const Mv& m, int only_accepted, int T, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, m.aff_n);
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
void launch_dlam(const Dev<R>& d, const Mv& m, R dl, hipStream_t st)
{
    hipLaunchKernelGGL(k_dlam<R>, dim3((m.aff_cap + 255) / 256), dim3(256), 0, st, d, m, dl);
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
void launch_kcnt(const Dev<R>& d, const Mv& m, int kind, hipStream_t st)
{
    hipLaunchKernelGGL(k_kcnt<R>, dim3(1), dim3(1024), 0, st, d, m, kind);
}

#define INSTM(R)                                                                         \
    template void launch_select<R>(const Dev<R>&, const Mv&, int, int, int, hipStream_t); \
    template void launch_mark<R>(const Dev<R>&, const Mv&, int, int, hipStream_t);        \
    template void launch_unmark<R>(const Dev<R>&, const Mv&, int, int, hipStream_t);      \
    template void launch_du<R>(const Dev<R>&, const Mv&, int, hipStream_t);               \
    template void launch_trial_accept<R>(const Dev<R>&, const Mv&, int, hipStream_t);     \
    template void launch_du_total<R>(const Dev<R>&, const Mv&, double*, hipStream_t);     \
    template void launch_aff_build<R>(const Dev<R>&, const Mv&, int, int, hipStream_t);   \
    template void launch_aff_clear<R>(const Dev<R>&, const Mv&, hipStream_t);             \
    template void launch_dforce<R>(const Dev<R>&, const Mv&, R, hipStream_t);             \
    template void launch_dlam<R>(const Dev<R>&, const Mv&, R, hipStream_t);               \
    template void launch_commit<R>(const Dev<R>&, const Mv&, int, int, hipStream_t);      \
    template void launch_mdas_accept<R>(const Dev<R>&, const Mv&, hipStream_t);           \
    template void launch_snapshot<R>(const Dev<R>&, const Mv&, int, hipStream_t);         \
    template void launch_kcnt<R>(const Dev<R>&, const Mv&, int, hipStream_t);
INSTM(float)
INSTM(double)

}  // namespace mbx
