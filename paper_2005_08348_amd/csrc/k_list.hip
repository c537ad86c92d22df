// k_list.hip -- cell binning (counting sort), periodic ghost images and the
// Verlet neighbour list.
//
// Layout.  Beads live in "slots" sorted by cell (cells of edge >= r_cut +
// skin, at least three per axis, z fastest), and within a cell by z, then
// bead id, so the order is deterministic and a bead's neighbours in a cell
// are nearby slots.  Coordinates stay in [0, L) up to the drift
// since the last rebuild.  Periodic images need no per-pair image
// arithmetic: the top cell layer of each axis is copied, shifted by -L
// (exact in floating point because x >= L/2), into a halo layer below 0
// ("ghost" slots N .. N+G), and a bead of the top layer that pairs with cell
// 0 across the face is itself shifted down by L (again exact).  A neighbour
// entry holds the slot j (real or ghost) and, for the entries that need it,
// three bits saying along which axes the i bead is shifted.  All resulting
// separations are single correctly rounded differences.
//
// Rebuild: binning, the cell layout (one work-group), scatter,
// per-cell sort and images, then the list build, one work-group per cell.
#include "membx_dev.h"

namespace mbx {

// ---------------------------------------------------------------- binning
constexpr int BB = 1024;   // threads per binning block and of the cell layout

// Extended grid: coordinate a in [0, nc] per axis, a = 0 is the halo layer
// holding images (shifted by -L) of real layer nc-1; a >= 1 is real cell a-1.
__device__ __forceinline__ void ext_coords(int e, const int ne[3], int a[3])
{
    a[2] = e % ne[2];
    a[1] = (e / ne[2]) % ne[1];
    a[0] = e / (ne[2] * ne[1]);
}

__device__ __forceinline__ int ext_source(const int a[3], const int nc[3])
{
    return ((a[0] ? a[0] - 1 : nc[0] - 1) * nc[1] + (a[1] ? a[1] - 1 : nc[1] - 1)) * nc[2] +
           (a[2] ? a[2] - 1 : nc[2] - 1);
}

// block-wide (BB threads) exclusive scan of per-thread values
__device__ __forceinline__ int block_scan(int v, int* sh)
{
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    int x = v;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const int y = __shfl_up(x, m);
        if (l >= m) x += y;
    }
    if (l == 63) sh[w] = x;
    __syncthreads();
    int base = 0;
    for (int q = 0; q < w; ++q) base += sh[q];
    __syncthreads();
    return base + x - v;
}

// Cell starts (exclusive scan of the counts), then the extended grid: real
// extended cells point into the slots, halo cells into the ghost range, laid
// out by a scan of their source cells' counts.  Each part is run by one
// work-group of BB threads, each taking a contiguous segment whose loads
// are all in flight at once (up to LU values per thread; longer segments in
// batches, read twice): the cell starts by k_layout (which also clears the
// counts for the next rebuild), the halo cells by an extra work-group of
// k_scatter, next to the scatter that needs only the cell starts.  LU is
// chosen per system at launch (8, or 64 and 16 for large grids): a batch
// wider than the segment costs instructions on small grids, a narrow one
// costs round trips on large ones.

// Halo cells in increasing extended index: the layer a0 = 0 (ne1 ne2 cells),
// then per a0 >= 1 the row a1 = 0 (ne2 cells) and the cells a1 >= 1, a2 = 0
// (ne1 - 1 cells).
__host__ __device__ __forceinline__ int halo_count(const int ne[3])
{
    return ne[1] * ne[2] + (ne[0] - 1) * (ne[2] + ne[1] - 1);
}
__device__ __forceinline__ int halo_ext(int h, const int ne[3])
{
    const int l0 = ne[1] * ne[2];
    if (h < l0) return h;
    const int g = ne[2] + ne[1] - 1, hh = h - l0;
    const int a0 = 1 + hh / g, r = hh - (a0 - 1) * g;
    const int a1 = r < ne[2] ? 0 : r - ne[2] + 1, a2 = r < ne[2] ? r : 0;
    return (a0 * ne[1] + a1) * ne[2] + a2;
}

template <typename R, int LU_L>
__device__ void layout_cells(const Dev<R>& d)
{
    __shared__ int sh[BB / 64];
    const int t = threadIdx.x;
    {
        const int per = (d.ncell + BB - 1) / BB;
        const int k0 = min(d.ncell, t * per), k1 = min(d.ncell, k0 + per);
        int v[LU_L];
        int s = 0;
        for (int kb = k0; kb < k1; kb += LU_L) {
#pragma unroll
            for (int u = 0; u < LU_L; ++u) v[u] = kb + u < k1 ? d.cell_cnt[kb + u] : 0;
#pragma unroll
            for (int u = 0; u < LU_L; ++u) s += v[u];
        }
        int run = block_scan(s, sh);
        for (int kb = k0; kb < k1; kb += LU_L) {
            if (per > LU_L) {   // segment longer than one batch: load again
#pragma unroll
                for (int u = 0; u < LU_L; ++u) v[u] = kb + u < k1 ? d.cell_cnt[kb + u] : 0;
            }
#pragma unroll
            for (int u = 0; u < LU_L; ++u)
                if (kb + u < k1) { d.cell_start[kb + u] = run; run += v[u]; }
        }
        if (t == BB - 1) d.cell_start[d.ncell] = run;
    }
    __syncthreads();
    for (int k = t; k < d.ncell; k += BB) d.cell_cnt[k] = 0;
}

// Halo cells of the extended grid (one work-group of BB threads): ghost
// ranges laid out by a scan of their source cells' counts, in increasing
// extended index.  Only halo cells are visited; the real extended cells are
// written by the scatter blocks.
template <typename R, int LU_H>
__device__ void layout_halo(const Dev<R>& d)
{
    __shared__ int sh[BB / 64];
    const int t = threadIdx.x;
    const int nh = halo_count(d.ne);
    const int per = (nh + BB - 1) / BB;
    const int k0 = min(nh, t * per), k1 = min(nh, k0 + per);
    int n[LU_H];
    auto fetch = [&](int kb) {
        int st[LU_H];
#pragma unroll
        for (int u = 0; u < LU_H; ++u) {
            st[u] = 0;
            n[u] = 0;
            if (kb + u < k1) {
                int a[3];
                ext_coords(halo_ext(kb + u, d.ne), d.ne, a);
                const int src = ext_source(a, d.nc);
                st[u] = d.cell_start[src];
                n[u] = d.cell_start[src + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < LU_H; ++u) n[u] -= st[u];
    };
    int s = 0;
    for (int kb = k0; kb < k1; kb += LU_H) {
        fetch(kb);
#pragma unroll
        for (int u = 0; u < LU_H; ++u) s += n[u];
    }
    int run = block_scan(s, sh);
    for (int kb = k0; kb < k1; kb += LU_H) {
        if (per > LU_H) fetch(kb);
#pragma unroll
        for (int u = 0; u < LU_H; ++u) {
            if (kb + u >= k1) continue;
            const int k = halo_ext(kb + u, d.ne);
            d.ext_start[k] = d.N + run;
            d.ext_cnt[k] = run >= d.Gcap ? 0 : min(n[u], d.Gcap - run);
            d.ext_scan[k] = run;          // ghost offset of this halo cell
            run += n[u];
        }
    }
    if (t == BB - 1) {
        *d.n_ghost = min(run, d.Gcap);
        if (run > d.Gcap) atomicOr(&d.flags[FL_GHOST_OVF], 1);
    }
}

// Bead -> cell for every slot, coordinates wrapped into [0, L) (bin_cell,
// bin_place); skipped when the force pass before the rebuild binned.
template <typename R>
__global__ __launch_bounds__(BB) void k_bin(Dev<R> d)
{
    const int i = blockIdx.x * BB + threadIdx.x;
    int cell = -1;
    if (i < d.N) {
        V4<R> p = d.posq[i];
        cell = bin_cell(d, p);
        d.posq[i] = p;
    }
    bin_place(d, i, cell);
}

template <typename R, int LU>
__global__ __launch_bounds__(BB) void k_layout(Dev<R> d)
{
    layout_cells<R, LU>(d);
}

// Scatter beads to their places in their cells' slot ranges (BB threads per
// block), and point the real extended cells at their slots; block 0,
// dispatched first as it is the longest, lays out the halo cells instead.
template <typename R, int LU>
__global__ __launch_bounds__(BB) void k_scatter(Dev<R> d)
{
    if (blockIdx.x == 0) {
        layout_halo<R, LU>(d);
        return;
    }
    const int g = (blockIdx.x - 1) * blockDim.x + threadIdx.x;
    const int stride = (gridDim.x - 1) * blockDim.x;
    for (int k = g; k < d.next; k += stride) {
        int a[3];
        ext_coords(k, d.ne, a);
        if (a[0] == 0 || a[1] == 0 || a[2] == 0) continue;
        const int src = ext_source(a, d.nc);
        const int st = d.cell_start[src];
        d.ext_start[k] = st;
        d.ext_cnt[k] = d.cell_start[src + 1] - st;
        d.ext_scan[k] = -1;
    }
    const int i = g;
    if (i >= d.N) return;
    const int dst = d.cell_start[d.cell_t[i]] + d.cell_pos[i];
    d.posq_t[dst] = d.posq[i];
    d.vel_t[dst] = d.vel[i];
    d.frc_t[dst] = d.frc[i];
    d.orig_t[dst] = d.orig[i];
    d.alch_t[dst] = d.alch[i];
}

// One wave per cell: the cell's beads in (z, bead id) order (a bead's rank is
// the number of the cell's beads with a smaller key) moved to their final slots,
// and their periodic images written to the halo cells this cell sources (the
// bead of rank r is image r of each); each bead records its images with
// their shift codes for the integrator.
// Sort key of a bead within its cell: the z coordinate's float32 bits (z is
// wrapped into [0, L), so the bits order like the values) above the bead id.
template <typename R>
__device__ __forceinline__ unsigned long long zkey(R z, int id)
{
    const float zf = (float)z;
    return ((unsigned long long)(unsigned)__float_as_int(zf) << 32) | (unsigned)id;
}

template <typename R>
__global__ __launch_bounds__(64) void k_place(Dev<R> d)
{
    __shared__ unsigned long long keys[256];
    const int cell = blockIdx.x, l = threadIdx.x;
    const int b = d.cell_start[cell], n = d.cell_start[cell + 1] - b;
    const int cz = cell % d.nc[2], cy = (cell / d.nc[2]) % d.nc[1], cx = cell / (d.nc[2] * d.nc[1]);
    const int top = (cx == d.nc[0] - 1 ? 1 : 0) | (cy == d.nc[1] - 1 ? 2 : 0) |
                    (cz == d.nc[2] - 1 ? 4 : 0);
    for (int m0 = 0; m0 < n; m0 += 64) {
        const int m = m0 + l;
        const int o = m < n ? d.orig_t[b + m] : 0x7fffffff;
        // the key: the wrapped z coordinate (non-negative, so its bits order
        // like the values) then the bead id; a strict total order
        const unsigned long long key =
            m < n ? zkey(d.posq_t[b + m].z, o) : ~0ull;
        int r = 0;
        for (int c0 = 0; c0 < n; c0 += 256) {
            const int nn = min(256, n - c0);
            __syncthreads();
            for (int k = l; k < nn; k += 64) keys[k] = zkey(d.posq_t[b + c0 + k].z, d.orig_t[b + c0 + k]);
            __syncthreads();
            for (int k = 0; k < nn; ++k) r += keys[k] < key ? 1 : 0;
        }
        if (m >= n) continue;
        const int p = b + m, s = b + r;
        const V4<R> x = d.posq_t[p];
        d.posq[s] = x;
        d.vel[s] = d.vel_t[p];
        d.frc[s] = d.frc_t[p];
        d.orig[s] = o;
        d.alch[s] = d.alch_t[p];
        d.inv[o] = s;
        d.orig_ext[s] = o;
        d.xref[s] = x;
        int4* gl = reinterpret_cast<int4*>(d.glist) + 2 * s;
        gl[0] = make_int4(-1, -1, -1, -1);
        gl[1] = make_int4(-1, -1, -1, -1);
        int q = 0;
        for (int code = 1; code < 8; ++code) {
            if (code & ~top) continue;
            const int e = (((code & 1) ? 0 : cx + 1) * d.ne[1] + ((code & 2) ? 0 : cy + 1)) * d.ne[2] +
                          ((code & 4) ? 0 : cz + 1);
            if (r < d.ext_cnt[e]) {   // else the ghost range is full (flagged)
                const int g = d.ext_scan[e] + r;
                V4<R> y = x;
                if (code & 1) y.x -= d.L[0];
                if (code & 2) y.y -= d.L[1];
                if (code & 4) y.z -= d.L[2];
                d.posq[d.N + g] = y;
                d.ghost_owner[g] = s;
                d.orig_ext[d.N + g] = o;
                d.glist[s * 8 + q] = g | (code << CODE_SHIFT);
            }
            ++q;
        }
    }
}


// ---------------------------------------------------------------- list
// exact float64 predicate d^2 < (r_cut + skin)^2, evaluated as
// ((dx*dx + dy*dy) + dz*dz) without contraction
__device__ __forceinline__ bool within_d(double xi, double yi, double zi, double xj, double yj,
                                         double zj, double rl2)
{
#pragma clang fp contract(off)
    double ex = xi - xj, ey = yi - yj, ez = zi - zj;
    double r2 = ex * ex;
    r2 = r2 + ey * ey;
    r2 = r2 + ez * ez;
    return r2 < rl2;
}

constexpr int LB = 256;   // threads per cell
constexpr int HS = 32;    // LDS candidate slots per lane (16-bit candidate indices)
constexpr int LU = 4;     // candidates per lane per round (LDS reads in flight)
template <typename R> struct CandCap { static constexpr int v = 1024; };
template <> struct CandCap<double> { static constexpr int v = 512; };

// Exact test of one entry: float64 from the stored coordinates, the i bead
// shifted down by L along the entry's code axes (exact), r^2 without
// contraction.
template <typename R>
__device__ __forceinline__ bool exact_in(const Dev<R>& d, const V4<R>& pi, int ent)
{
    const int j = ent & JMASK, code = (int)((unsigned)ent >> CODE_SHIFT);
    const V4<R> pj = d.posq[j];
    const R xs = (code & 1) ? pi.x - d.L[0] : pi.x;
    const R ys = (code & 2) ? pi.y - d.L[1] : pi.y;
    const R zs = (code & 4) ? pi.z - d.L[2] : pi.z;
    return within_d((double)xs, (double)ys, (double)zs, (double)pj.x, (double)pj.y, (double)pj.z,
                    d.rl2d);
}

template <typename R>
__device__ __forceinline__ R img_r2(const V4<R>& pi, const V4<R>& pj)
{
    const R dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    return dx * dx + dy * dy + dz * dz;
}

// One candidate: prefilter in R on the candidate image stored in LDS (the j
// bead shifted UP by L along the code axes, rounded): below rl2_lo a hit,
// above rl2_hi a miss, the band in between decided exactly.  Bonded partners
// and the bead itself are excluded through the bead's exclusion mask (bit
// 16 + class - bead id; the 64-bit shift reads zero beyond bit 31).  The band
// is many ulps wide, so the decision does not depend on how r^2 was rounded.
__device__ __forceinline__ bool excluded(unsigned long long exm, int rel)
{
    return (exm >> min((unsigned)rel, 63u)) & 1ull;
}

template <typename R>
__device__ __forceinline__ bool cand_in(const Dev<R>& d, const V4<R>& pi, int oi16,
                                        unsigned long long exm, const V4<R>& pj, int ent)
{
    const R r2 = img_r2(pi, pj);
    bool in = r2 < d.rl2_lo;
    if (!in && !(r2 > d.rl2_hi)) in = exact_in(d, pi, ent);
    return in && !excluded(exm, cls_of<R>(pj.w) + oi16);
}

// List build, one work-group per cell.  The candidates of the 27 neighbour
// cells are staged in LDS (image position, bead id, entry = slot | code << 29
// with code the axes along which the i bead is shifted), followed by a
// sentinel that never hits; each bead of the cell owns Q lanes that split
// the candidates (lane q takes q, q + Q, ...).  Per staging round every lane
// tests its candidates once (the rare band cases exactly, in a wave-uniform
// branch) and notes the hits in its LDS buffer as 16-bit candidate indices;
// lane q of bead i then writes its entries after lanes 0..q-1 and after the
// earlier rounds, so the lists are deterministic.  A lane whose buffer
// overflows (very crowded cells) tests its candidates again while writing.
template <typename R>
__global__ __launch_bounds__(LB) void k_list(Dev<R> d)
{
    constexpr int CMAX = CandCap<R>::v;
    constexpr int NW = LB / 64;
    constexpr int HP = HS + 4;   // buffer pitch (8-byte aligned rows)
    __shared__ V4<R> cpos[CMAX + 1];
    __shared__ int cjs[CMAX + 1];
    __shared__ __align__(8) unsigned short hits[LB * HP];
    __shared__ int off[28], jst[27], cod[27];
    __shared__ int cnt[LB];
    const int cell = xcd_block(blockIdx.x, gridDim.x);
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int Kc = d.Kcap;
    const int s0 = d.cell_start[cell], ni = d.cell_start[cell + 1] - s0;
    if (ni == 0) return;
    // bonded terms of the cell's beads with their partners' slots
    for (int k = t; k < ni * MAXBT; k += LB) {
        const int i = s0 + k / MAXBT, tt = k % MAXBT;
        const int o = d.orig[i];
        const int b0 = d.bt_off[o], n = d.bt_off[o + 1] - b0;
        int4 e = make_int4(-1, i, i, 0);
        if (tt < n) {
            const int4 tm = d.bt[b0 + tt];
            e = make_int4(tm.x, d.inv[tm.y], tm.z >= 0 ? d.inv[tm.z] : i, tm.w);
        }
        d.bslot[(size_t)i * MAXBT + tt] = e;
    }
    if (w == 0) {
        const int cz = cell % d.nc[2], cy = (cell / d.nc[2]) % d.nc[1], cx = cell / (d.nc[2] * d.nc[1]);
        int n = 0;
        if (l < 27) {
            const int ox = l / 9 - 1, oy = (l / 3) % 3 - 1, oz = l % 3 - 1;
            int ax = cx + ox, ay = cy + oy, az = cz + oz, code = 0;
            if (ax == d.nc[0]) { ax = 0; code |= 1; }
            if (ay == d.nc[1]) { ay = 0; code |= 2; }
            if (az == d.nc[2]) { az = 0; code |= 4; }
            const int e = ((ax + 1) * d.ne[1] + (ay + 1)) * d.ne[2] + (az + 1);
            jst[l] = d.ext_start[e];
            cod[l] = code;
            n = d.ext_cnt[e];
        }
#pragma unroll
        for (int m = 1; m < 32; m <<= 1) {
            const int y = __shfl_up(n, m);
            if (l >= m) n += y;
        }
        if (l < 27) off[l + 1] = n;
        if (l == 0) off[0] = 0;
    }
    __syncthreads();
    const int C = off[27];
    const bool one_round = C <= CMAX;
    // staging: wave w takes cells w, w + NW, ..., one candidate per lane
    // (loads of all its cells in flight), cells above 64 candidates looped
    auto stage = [&](int cb, int nc) {
        __syncthreads();
        constexpr int NU = (27 + NW - 1) / NW;
        int js[NU], dst[NU], cs[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int o = w + u * NW;
            dst[u] = -1; js[u] = 0; cs[u] = 0;
            if (o < 27) {
                const int lo = max(off[o], cb), hi = min(off[o + 1], cb + nc);
                if (lo + l < hi) {
                    dst[u] = lo + l - cb;
                    js[u] = jst[o] + (lo + l - off[o]);
                    cs[u] = cod[o];
                }
            }
        }
        V4<R> ps[NU];
        int oj[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) { ps[u] = d.posq[js[u]]; oj[u] = d.orig_ext[js[u]]; }
        auto put = [&](int c, V4<R> p, int code, int oo, int j) {
            if (code & 1) p.x += d.L[0];
            if (code & 2) p.y += d.L[1];
            if (code & 4) p.z += d.L[2];
            p.w = cls_to<R>(oo);
            cpos[c] = p;
            cjs[c] = j | (code << CODE_SHIFT);
        };
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (dst[u] >= 0) put(dst[u], ps[u], cs[u], oj[u], js[u]);
        for (int o = w; o < 27; o += NW) {
            const int lo = max(off[o], cb), hi = min(off[o + 1], cb + nc);
            for (int idx = lo + 64 + l; idx < hi; idx += 64) {
                const int j = jst[o] + (idx - off[o]);
                put(idx - cb, d.posq[j], cod[o], d.orig_ext[j], j);
            }
        }
        if (t == 0) {
            const R far = (R)1e15;
            cpos[nc] = V4<R>{ far, far, far, cls_to<R>(-(1 << 20)) };
            cjs[nc] = 0;
        }
        __syncthreads();
    };
    for (int ib = 0; ib < ni; ib += LB) {
        const int nib = min(LB, ni - ib);
        const int Q = max(1, LB / nib);
        const int li = t / Q, q = t % Q;
        const bool act = li < nib;
        const int i = s0 + ib + (act ? li : 0);
        const V4<R> pi = d.posq[i];
        const int oi16 = 16 - d.orig[i];
        const unsigned long long exm = d.exmask[d.orig[i]];
        const size_t ibase = nbr_base(i, Kc, d.lpb_shift, d.bg_shift);
        unsigned short* hb = hits + t * HP;
        int kb = 0;   // entries of bead i written by earlier rounds
        for (int cb = 0; cb < C; cb += CMAX) {
            const int nc = min(CMAX, C - cb);
            if (!(one_round && ib > 0)) stage(cb, nc);
            const int nu = (nc + Q - 1) / Q;
            const int q0 = act ? q : nc;   // idle lanes read the sentinel only
            // every candidate is written to the next free slot (slot HS once
            // full); the count advances on a hit
            int nh = 0;
            const R lo2 = d.rl2_lo, hi2 = d.rl2_hi;
            for (int u0 = 0; u0 < nu; u0 += LU) {
                int cc[LU];
                V4<R> pj[LU];
#pragma unroll
                for (int k = 0; k < LU; ++k) {
                    cc[k] = min(q0 + (u0 + k) * Q, nc);
                    pj[k] = cpos[cc[k]];
                }
                bool in[LU];
                unsigned bm = 0;   // candidates in the band
#pragma unroll
                for (int k = 0; k < LU; ++k) {
                    const R r2 = img_r2(pi, pj[k]);
                    const bool ex = excluded(exm, cls_of<R>(pj[k].w) + oi16);
                    in[k] = !(r2 > hi2) & !ex;
                    bm |= (unsigned)(in[k] & !(r2 < lo2)) << k;
                }
                if (__builtin_expect(__any(bm != 0), 0)) {
#pragma unroll
                    for (int k = 0; k < LU; ++k)
                        if ((bm >> k) & 1u) in[k] = exact_in(d, pi, cjs[cc[k]]);
                }
#pragma unroll
                for (int k = 0; k < LU; ++k) {
                    hb[min(nh, HS)] = (unsigned short)cc[k];
                    nh += in[k] ? 1 : 0;
                }
            }
            cnt[t] = act ? nh : 0;
            __syncthreads();
            int b0 = 0, tot = 0;
            if (act)
                for (int qq = 0; qq < Q; ++qq) {
                    const int c0 = cnt[li * Q + qq];
                    if (qq < q) b0 += c0;
                    tot += c0;
                }
            if (act) {
                const int k0 = kb + b0;
                if (nh <= HS) {
                    // four entries per round: buffer word, then their entries
                    for (int k = 0; k < nh; k += 4) {
                        const uint2 hw = *reinterpret_cast<const uint2*>(hb + k);
                        const int c4[4] = { (int)(hw.x & 0xffff), (int)(hw.x >> 16),
                                            (int)(hw.y & 0xffff), (int)(hw.y >> 16) };
                        int e4[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) e4[u] = cjs[min(c4[u], nc)];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (k + u < nh && k0 + k + u < Kc)
                                d.nbr[ibase + nbr_koff(k0 + k + u, d.lpb_shift)] = e4[u];
                    }
                } else {
                    atomicOr(&d.flags[FL_HIT_OVF], 1);
                    int mm = 0;
                    for (int u = 0; u < nu; ++u) {
                        const int c = q + u * Q;
                        if (!(c < nc && cand_in(d, pi, oi16, exm, cpos[c], cjs[c]))) continue;
                        const int k = k0 + mm++;
                        if (k < Kc) d.nbr[ibase + nbr_koff(k, d.lpb_shift)] = cjs[c];
                    }
                }
            }
            kb += tot;
            __syncthreads();   // cnt, the buffers and the staged candidates are reused
        }
        if (act && q == 0) {
            d.nseg0[i] = 0;
            d.ncnt[i] = min(kb, Kc);
            if (kb > Kc) {
                atomicOr(&d.flags[FL_LIST_OVF], 1);
                atomicMax(&d.flags[FL_LIST_NEED], kb);
            }
        }
    }
}

// ----------------------------------------------------------------- launch
#define GRID(n) dim3(((n) + WG - 1) / WG), dim3(WG)

template <typename R>
void launch_rebuild(const Dev<R>& d, hipStream_t st, bool binned)
{
    if (!binned) hipLaunchKernelGGL(k_bin<R>, dim3((d.N + BB - 1) / BB), dim3(BB), 0, st, d);
    // segment lengths of the two single-work-group scans
    const int per_c = (d.ncell + BB - 1) / BB;
    const int per_h = (halo_count(d.ne) + BB - 1) / BB;
    if (per_c <= 8) hipLaunchKernelGGL((k_layout<R, 8>), dim3(1), dim3(BB), 0, st, d);
    else hipLaunchKernelGGL((k_layout<R, 64>), dim3(1), dim3(BB), 0, st, d);
    if (per_h <= 8)
        hipLaunchKernelGGL((k_scatter<R, 8>), dim3((d.N + BB - 1) / BB + 1), dim3(BB), 0, st, d);
    else
        hipLaunchKernelGGL((k_scatter<R, 16>), dim3((d.N + BB - 1) / BB + 1), dim3(BB), 0, st, d);
    hipLaunchKernelGGL(k_place<R>, dim3(d.ncell), dim3(64), 0, st, d);
    hipLaunchKernelGGL(k_list<R>, dim3(d.ncell), dim3(LB), 0, st, d);
}


template void launch_rebuild<float>(const Dev<float>&, hipStream_t, bool);
template void launch_rebuild<double>(const Dev<double>&, hipStream_t, bool);

}  // namespace mbx
