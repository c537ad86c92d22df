// k_list.hip -- cell binning (counting sort), periodic ghost images and the
// Verlet neighbour list.
//
// Layout.  Beads live in "slots" sorted by cell (cells of edge >= r_cut +
// skin, at least three per axis), and within a cell by bead id, so the sort
// is deterministic.  Coordinates stay in [0, L) up to the drift since the
// last rebuild.  Periodic images are handled without any per-pair image
// arithmetic: the top cell layer of each axis is copied, shifted by -L
// (exact in floating point because x >= L/2), into a halo layer below 0
// ("ghost" slots N.. N+G), and a bead of the top layer that pairs with cell
// 0 across the face is itself shifted down by L (again exact).  A neighbour
// entry therefore holds the slot j (real or ghost) and, for the rare entries
// that need it, three bits saying along which axes the i bead is shifted.
// All resulting separations are single correctly rounded differences.
#include "membx_dev.h"

namespace mbx {

// ---------------------------------------------------------------- binning
template <typename R>
__global__ void k_bin(Dev<R> d)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    V4<R> p = d.posq[i];
    R* c[3] = { &p.x, &p.y, &p.z };
    int cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R x = *c[a];
        if (x >= d.L[a]) x -= d.L[a];        // exact (Sterbenz) for x in [L, 2L]
        else if (x < (R)0) x += d.L[a];
        if (!(x >= (R)0 && x < d.L[a])) {     // far outside (set_state, minimizer)
            double xd = (double)*c[a];
            xd -= d.Ld[a] * floor(xd / d.Ld[a]);
            x = (R)xd;
            if (x >= d.L[a]) x = (R)0;
        }
        *c[a] = x;
        int ci = (int)(x * d.inv_edge[a]);
        cc[a] = ci < 0 ? 0 : (ci >= d.nc[a] ? d.nc[a] - 1 : ci);
    }
    d.posq[i] = p;
    int cell = (cc[0] * d.nc[1] + cc[1]) * d.nc[2] + cc[2];
    d.cell_t[i] = cell;
    atomicAdd(&d.cell_cnt[cell], 1);
}

// Exclusive scan of in[0..n) into out[0..n], out[n] = total; one work-group.
__global__ void k_scan(const int* __restrict__ in, int* __restrict__ out, int n)
{
    __shared__ int part[1024];
    int t = threadIdx.x;
    int per = (n + 1023) / 1024;
    int b = t * per, e = min(n, b + per);
    int s = 0;
    for (int k = b; k < e; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int k = b; k < e; ++k) { out[k] = run; run += in[k]; }
    if (t == 1023) out[n] = part[1023];
}

// Scatter beads to their cell ranges (arbitrary order inside a cell).
template <typename R>
__global__ void k_scatter(Dev<R> d)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    int c = d.cell_t[i];
    int dst = d.cell_start[c] + atomicAdd(&d.cell_cur[c], 1);
    d.posq_t[dst] = d.posq[i];
    d.vel_t[dst] = d.vel[i];
    d.frc_t[dst] = d.frc[i];
    d.orig_t[dst] = d.orig[i];
    d.alch_t[dst] = d.alch[i];
}

// Order each cell by bead id: a bead's final slot is the cell start plus the
// number of beads of its cell with a smaller id.
template <typename R>
__global__ void k_rank(Dev<R> d)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.N) return;
    int o = d.orig_t[p];
    V4<R> x = d.posq_t[p];
    int cell = -1;
    // find the cell of tmp position p: binary search in cell_start
    int lo = 0, hi = d.ncell;   // cell_start[lo] <= p < cell_start[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (d.cell_start[mid] <= p) lo = mid; else hi = mid;
    }
    cell = lo;
    int b = d.cell_start[cell], e = d.cell_start[cell + 1];
    int r = 0;
    for (int q = b; q < e; ++q) r += d.orig_t[q] < o;
    int s = b + r;
    d.posq[s] = x;
    d.vel[s] = d.vel_t[p];
    d.frc[s] = d.frc_t[p];
    d.orig[s] = o;
    d.alch[s] = d.alch_t[p];
    d.cellid[s] = cell;
    d.inv[o] = s;
    d.xref[s] = x;
}

// ----------------------------------------------------------------- ghosts
// Extended grid: coordinate a in [0, nc] per axis, a = 0 is the halo layer
// holding images (shifted by -L) of real layer nc-1; a >= 1 is real cell a-1.
__device__ __forceinline__ void ext_coords(int e, const int ne[3], int a[3])
{
    a[2] = e % ne[2];
    a[1] = (e / ne[2]) % ne[1];
    a[0] = e / (ne[2] * ne[1]);
}

template <typename R>
__global__ void k_ghost_count(Dev<R> d)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d.next) return;
    int a[3];
    ext_coords(e, d.ne, a);
    int halo = (a[0] == 0) | (a[1] == 0) | (a[2] == 0);
    int src[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) src[k] = a[k] == 0 ? d.nc[k] - 1 : a[k] - 1;
    int rc = (src[0] * d.nc[1] + src[1]) * d.nc[2] + src[2];
    d.ext_cnt[e] = d.cell_cnt[rc];
    d.ext_start[e] = halo ? 0 : d.cell_start[rc];
    // halo counts feed the ghost scan; real cells contribute nothing
    d.ext_scan[e] = halo ? d.cell_cnt[rc] : 0;
}

template <typename R>
__global__ void k_ghost_fill(Dev<R> d, const int* __restrict__ goff)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        int tot = goff[d.next];
        *d.n_ghost = tot < d.Gcap ? tot : d.Gcap;
        if (tot > d.Gcap) atomicOr(&d.flags[FL_GHOST_OVF], 1);
    }
    if (e >= d.next) return;
    int a[3];
    ext_coords(e, d.ne, a);
    int code = (a[0] == 0 ? 1 : 0) | (a[1] == 0 ? 2 : 0) | (a[2] == 0 ? 4 : 0);
    if (!code) return;
    int src[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) src[k] = a[k] == 0 ? d.nc[k] - 1 : a[k] - 1;
    int rc = (src[0] * d.nc[1] + src[1]) * d.nc[2] + src[2];
    int s0 = d.cell_start[rc], n = d.cell_cnt[rc];
    int g0 = goff[e];
    d.ext_start[e] = d.N + g0;
    int nfit = n;
    if (g0 + n > d.Gcap) nfit = d.Gcap > g0 ? d.Gcap - g0 : 0;
    d.ext_cnt[e] = nfit;
    for (int k = 0; k < nfit; ++k) {
        int g = g0 + k, s = s0 + k;
        V4<R> p = d.posq[s];
        if (code & 1) p.x -= d.L[0];
        if (code & 2) p.y -= d.L[1];
        if (code & 4) p.z -= d.L[2];
        d.posq[d.N + g] = p;
        d.ghost_owner[g] = s;
        d.ghost_code[g] = code;
    }
}

// Refresh ghost coordinates (and class) from their owners after a move.
template <typename R>
__global__ void k_ghost_update(Dev<R> d)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= *d.n_ghost) return;
    int s = d.ghost_owner[g], code = d.ghost_code[g];
    V4<R> p = d.posq[s];
    if (code & 1) p.x -= d.L[0];
    if (code & 2) p.y -= d.L[1];
    if (code & 4) p.z -= d.L[2];
    d.posq[d.N + g] = p;
}

// ---------------------------------------------------------------- list
template <typename R>
__device__ __forceinline__ bool within_rlist(const Dev<R>& d, R dx, R dy, R dz, double xi,
                                             double yi, double zi, const V4<R>& pj)
{
    // exact float64 predicate d^2 < (r_cut + skin)^2, evaluated as
    // ((dx*dx + dy*dy) + dz*dz) without contraction
#pragma clang fp contract(off)
    double ex = xi - (double)pj.x, ey = yi - (double)pj.y, ez = zi - (double)pj.z;
    double r2 = ex * ex;
    r2 = r2 + ey * ey;
    r2 = r2 + ez * ez;
    return r2 < d.rl2d;
}

template <typename R>
__global__ __launch_bounds__(WG) void k_list(Dev<R> d)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    V4<R> pi = d.posq[i];
    int cell = d.cellid[i];
    int cz = cell % d.nc[2], cy = (cell / d.nc[2]) % d.nc[1], cx = cell / (d.nc[2] * d.nc[1]);
    int oi = d.orig[i];
    int ex[MAXEXCL];
#pragma unroll
    for (int e = 0; e < MAXEXCL; ++e) ex[e] = d.excl[oi * MAXEXCL + e];
    int k = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int o = 0; o < 27; ++o) {
            int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
            int ax = cx + ox, ay = cy + oy, az = cz + oz, code = 0;
            if (ax == d.nc[0]) { ax = 0; code |= 1; }
            if (ay == d.nc[1]) { ay = 0; code |= 2; }
            if (az == d.nc[2]) { az = 0; code |= 4; }
            if ((pass == 0) != (code == 0)) continue;
            int e = ((ax + 1) * d.ne[1] + (ay + 1)) * d.ne[2] + (az + 1);
            int j0 = d.ext_start[e], jn = d.ext_cnt[e];
            R xs = pi.x, ys = pi.y, zs = pi.z;
            if (code & 1) xs -= d.L[0];
            if (code & 2) ys -= d.L[1];
            if (code & 4) zs -= d.L[2];
            double xd = (double)xs, yd = (double)ys, zd = (double)zs;
            for (int j = j0; j < j0 + jn; ++j) {
                if (j == i) continue;
                V4<R> pj = d.posq[j];
                R dx = xs - pj.x, dy = ys - pj.y, dz = zs - pj.z;
                bool in;
                if (sizeof(R) == 4) {
                    float r2f = (float)(dx * dx + dy * dy + dz * dz);
                    if (r2f < d.rl2f_lo) in = true;
                    else if (r2f > d.rl2f_hi) in = false;
                    else in = within_rlist(d, dx, dy, dz, xd, yd, zd, pj);
                } else {
                    in = within_rlist(d, dx, dy, dz, xd, yd, zd, pj);
                }
                if (!in) continue;
                int oj = j < d.N ? d.orig[j] : d.orig[d.ghost_owner[j - d.N]];
                bool exc = false;
#pragma unroll
                for (int q = 0; q < MAXEXCL; ++q) exc |= (ex[q] == oj);
                if (exc) continue;
                if (k < d.Kcap) d.nbr[(size_t)k * d.Npad + i] = j | (code << CODE_SHIFT);
                ++k;
            }
        }
        if (pass == 0) d.nseg0[i] = min(k, d.Kcap);
    }
    if (k > d.Kcap) atomicOr(&d.flags[FL_LIST_OVF], 1);
    d.ncnt[i] = min(k, d.Kcap);
}

// ----------------------------------------------------------------- launch
#define GRID(n) dim3(((n) + WG - 1) / WG), dim3(WG)

template <typename R>
void launch_rebuild(const Dev<R>& d, hipStream_t st)
{
    // zero counters with a fill kernel (no memset nodes in captured graphs)
    extern void launch_fill_i32(int* p, int v, size_t n, hipStream_t st);
    launch_fill_i32(d.cell_cnt, 0, d.ncell, st);
    launch_fill_i32(d.cell_cur, 0, d.ncell, st);
    hipLaunchKernelGGL(k_bin<R>, GRID(d.N), 0, st, d);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d.cell_cnt, d.cell_start, d.ncell);
    hipLaunchKernelGGL(k_scatter<R>, GRID(d.N), 0, st, d);
    hipLaunchKernelGGL(k_rank<R>, GRID(d.N), 0, st, d);
    hipLaunchKernelGGL(k_ghost_count<R>, GRID(d.next), 0, st, d);
    // ghost offsets: scan of the halo counts (in place into cell_cur-free scratch)
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d.ext_scan, d.ext_scan + d.next + 1,
                       d.next);
    hipLaunchKernelGGL(k_ghost_fill<R>, GRID(d.next), 0, st, d,
                       (const int*)(d.ext_scan + d.next + 1));
    hipLaunchKernelGGL(k_list<R>, GRID(d.N), 0, st, d);
}

template <typename R>
void launch_ghost_update(const Dev<R>& d, hipStream_t st)
{
    hipLaunchKernelGGL(k_ghost_update<R>, GRID(d.Gcap), 0, st, d);
}

template void launch_rebuild<float>(const Dev<float>&, hipStream_t);
template void launch_rebuild<double>(const Dev<double>&, hipStream_t);
template void launch_ghost_update<float>(const Dev<float>&, hipStream_t);
template void launch_ghost_update<double>(const Dev<double>&, hipStream_t);

}  // namespace mbx
