// re_kernels.hip -- gfx950 kernels of the replica-exchange LJ engine.
//
// Two precision policies share one set of kernel templates:
//   PMixed: positions are 32-bit periodic fixed point (one int32 per
//           coordinate spans the box, so integer wraparound is the minimum
//           image and the cell index is an exact integer product), pair
//           vectors are converted to FP32 in grid units; velocities and
//           forces FP32; the per-replica energy sum and all exchange
//           arithmetic are FP64.
//   PF64:   FP64 positions (explicit minimum image), velocities and forces.
//
// The step is BAOAB Langevin dynamics (velocity-Verlet core) on a Verlet
// neighbour list to r_c + skin, updated when one atom moved more than
// skin/2 since the last update (Example section).  Temperatures move
// between replicas by the Metropolis rule (Implementation section).
#include "re_internal.hpp"

namespace re {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications by the Philox multipliers, the high halves mixed
// with the odd counter words and the round key; the key advances by the two
// Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    return philox10(make_uint4(c0, c1, c2, c3), (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Box-Muller (Box & Muller 1958): words 0,1 -> cos/sin pair, words 2,3 -> cos.
// FP32 version takes the top 24 bits of each word: u = (w>>8 + 1/2) 2^-24.
__device__ __forceinline__ void normals3f(uint4 w, float& z0, float& z1, float& z2)
{
    const float u0 = ((float)(w.x >> 8) + 0.5f) * 0x1p-24f;
    const float u1 = ((float)(w.y >> 8) + 0.5f) * 0x1p-24f;
    const float u2 = ((float)(w.z >> 8) + 0.5f) * 0x1p-24f;
    const float u3 = ((float)(w.w >> 8) + 0.5f) * 0x1p-24f;
    const float r01 = __fsqrt_rn(-2.0f * __logf(u0));
    const float r23 = __fsqrt_rn(-2.0f * __logf(u2));
    float s1, c1;
    __sincosf(6.28318530717958648f * u1, &s1, &c1);
    z0 = r01 * c1;
    z1 = r01 * s1;
    z2 = r23 * __cosf(6.28318530717958648f * u3);
}

// FP64 version: u = (w + 1/2) 2^-32.
__device__ __forceinline__ void normals3d(uint4 w, double& z0, double& z1, double& z2)
{
    const double u0 = ((double)w.x + 0.5) * 0x1p-32;
    const double u1 = ((double)w.y + 0.5) * 0x1p-32;
    const double u2 = ((double)w.z + 0.5) * 0x1p-32;
    const double u3 = ((double)w.w + 0.5) * 0x1p-32;
    const double two_pi = 6.283185307179586476925286766559;
    const double r01 = sqrt(-2.0 * log(u0));
    const double r23 = sqrt(-2.0 * log(u2));
    z0 = r01 * cos(two_pi * u1);
    z1 = r01 * sin(two_pi * u1);
    z2 = r23 * cos(two_pi * u3);
}

// 53-bit uniform of exchange attempt k for the lower replica id.
__device__ __forceinline__ double uniform53(uint64_t seed, int64_t k, int32_t lower)
{
    const uint4 w = draw(seed, (uint32_t)(uint64_t)k, (uint32_t)((uint64_t)k >> 32), (uint32_t)lower, kPurposeExchange);
    const uint64_t m = ((uint64_t)(w.x >> 5) << 26) | (uint64_t)(w.y >> 6);
    return (double)m * 0x1p-53;
}

// ---------------------------------------------------------------------------
// Precision policies.
struct PMixed {
    using pos_t = int4;
    using vel_t = float4;
    using real = float;
    static constexpr bool kF64 = false;
    __device__ static pos_t* pos(const DevState& d, int b) { return d.posi[b]; }
    __device__ static vel_t* vel(const DevState& d) { return d.velf; }
    __device__ static vel_t* velt(const DevState& d) { return d.veltf; }
    __device__ static vel_t* frc(const DevState& d) { return d.frcf; }
    __device__ static pos_t* xref(const DevState& d) { return d.xrefi; }
    __device__ static real* epot(const DevState& d) { return d.epotf; }
    __device__ static int id(const pos_t& p) { return p.w; }
    __device__ static int wrapdiff(int a, int b) { return (int)((uint32_t)a - (uint32_t)b); }
    // pair vector a - b in grid units (the wraparound is the minimum image)
    __device__ static void diff(const pos_t& a, const pos_t& b, const RepDev&, real& dx, real& dy, real& dz)
    {
        dx = (float)wrapdiff(a.x, b.x);
        dy = (float)wrapdiff(a.y, b.y);
        dz = (float)wrapdiff(a.z, b.z);
    }
    // x += h v: the displacement rounded to the grid; wraps by itself
    __device__ static pos_t drift(pos_t p, real hx, real hy, real hz, const RepDev& rd)
    {
        p.x = (int)((uint32_t)p.x + (uint32_t)__float2int_rn(hx * rd.inv_sf));
        p.y = (int)((uint32_t)p.y + (uint32_t)__float2int_rn(hy * rd.inv_sf));
        p.z = (int)((uint32_t)p.z + (uint32_t)__float2int_rn(hz * rd.inv_sf));
        return p;
    }
    __device__ static int cellc(int x, const RepDev& rd)
    {
        return (int)__umulhi((uint32_t)x ^ 0x80000000u, (uint32_t)rd.ncell);
    }
    __device__ static real rc2(const RepDev& rd) { return rd.rc2f; }
    __device__ static real rl2(const RepDev& rd) { return rd.rl2f; }
    __device__ static real lim2(const RepDev& rd) { return rd.lim2f; }
};

struct PF64 {
    using pos_t = double4;
    using vel_t = double4;
    using real = double;
    static constexpr bool kF64 = true;
    __device__ static pos_t* pos(const DevState& d, int b) { return d.posd[b]; }
    __device__ static vel_t* vel(const DevState& d) { return d.veld; }
    __device__ static vel_t* velt(const DevState& d) { return d.veltd; }
    __device__ static vel_t* frc(const DevState& d) { return d.frcd; }
    __device__ static pos_t* xref(const DevState& d) { return d.xrefd; }
    __device__ static real* epot(const DevState& d) { return d.epotd; }
    __device__ static int id(const pos_t& p) { return (int)p.w; }
    __device__ static double mi(double x, const RepDev& rd) { return x - rd.L * rint(x / rd.L); }
    __device__ static void diff(const pos_t& a, const pos_t& b, const RepDev& rd, real& dx, real& dy, real& dz)
    {
        dx = mi(a.x - b.x, rd);
        dy = mi(a.y - b.y, rd);
        dz = mi(a.z - b.z, rd);
    }
    __device__ static double wrap(double x, const RepDev& rd) { return x - rd.L * floor((x + 0.5 * rd.L) / rd.L); }
    __device__ static pos_t drift(pos_t p, real hx, real hy, real hz, const RepDev& rd)
    {
        p.x = wrap(p.x + hx, rd);
        p.y = wrap(p.y + hy, rd);
        p.z = wrap(p.z + hz, rd);
        return p;
    }
    __device__ static int cellc(double x, const RepDev& rd)
    {
        int c = (int)floor((x / rd.L + 0.5) * (double)rd.ncell);
        return c < 0 ? 0 : (c >= rd.ncell ? rd.ncell - 1 : c);
    }
    __device__ static real rc2(const RepDev& rd) { return rd.rc2d; }
    __device__ static real rl2(const RepDev& rd) { return rd.rl2d; }
    __device__ static real lim2(const RepDev& rd) { return rd.lim2d; }
};

template <class P>
__device__ __forceinline__ void set_xyz(typename P::vel_t& v, typename P::real x, typename P::real y, typename P::real z)
{
    v.x = x;
    v.y = y;
    v.z = z;
}

// ---------------------------------------------------------------------------
// First half of a step from a stopped boundary (B A O A of BAOAB), for every
// atom of the block's replica:  v = alpha v + h F;  x += h v;
// v = c1 v + c2 xi;  x += h v;  then the half-skin test against xref.
template <class P>
__global__ __launch_bounds__(256) void k_start(DevState d, StepArgs sa)
{
    using real = typename P::real;
    const int cur = sa.cur, R = sa.R;
    const int64_t step = sa.step;
    const int b = sa.blk_off + blockIdx.x;
    const int r = sa.tab.rep[b];
    if (r < 0) return;
    const RepDev rd = d.rep[r];
    const int i = sa.tab.a0[b] + threadIdx.x;
    if (i >= rd.N) return;
    const int g = rd.base + i;
    typename P::pos_t* pos = P::pos(d, cur);
    typename P::pos_t x = pos[g];
    typename P::vel_t v = P::vel(d)[g];
    const typename P::vel_t f = P::frc(d)[g];
    const real hh = (real)sa.h;
    const real a = sa.apply_alpha ? (real)d.alpha[r] : (real)1;
    const real c1 = (real)sa.c1;
    const real c2 = (real)d.c2[r];
    real vx = a * v.x + hh * f.x, vy = a * v.y + hh * f.y, vz = a * v.z + hh * f.z;
    x = P::drift(x, hh * vx, hh * vy, hh * vz, rd);
    const uint4 w = draw(sa.seed, (uint32_t)P::id(x), (uint32_t)step, (uint32_t)r, kPurposeOStep);
    real z0, z1, z2;
    if constexpr (P::kF64) {
        normals3d(w, z0, z1, z2);
    } else {
        normals3f(w, z0, z1, z2);
    }
    vx = c1 * vx + c2 * z0;
    vy = c1 * vy + c2 * z1;
    vz = c1 * vz + c2 * z2;
    x = P::drift(x, hh * vx, hh * vy, hh * vz, rd);
    pos[g] = x;
    set_xyz<P>(v, vx, vy, vz);
    P::vel(d)[g] = v;
    real dx, dy, dz;
    P::diff(x, P::xref(d)[g], rd, dx, dy, dz);
    if (dx * dx + dy * dy + dz * dz > P::lim2(rd)) atomicOr(&d.flag[(size_t)((step + 1) & 1) * R + r], 1u);
}

// ---------------------------------------------------------------------------
// Reorder one replica by cell (one workgroup per replica): counting sort of
// the atoms into the cell grid, each cell ordered by atom id so the result is
// independent of scheduling; x_ref := x.  Runs only for replicas whose
// update flag of this parity is set (or all, when force_all).
template <class P>
__global__ __launch_bounds__(kReorderThreads) void k_reorder(DevState d, StepArgs sa)
{
    const int cur = sa.cur, par = sa.par, R = sa.R, force_all = sa.force_all;
    const int r = sa.r0 + blockIdx.x;
    if (!force_all && d.flag[(size_t)par * R + r] == 0) return;
    const RepDev rd = d.rep[r];
    __shared__ int cnt[kMaxCells + 1];
    __shared__ int part[kReorderThreads];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nc = rd.ncell, ncc = nc * nc * nc;
    typename P::pos_t* pos = P::pos(d, cur) + rd.base;
    typename P::pos_t* tmp = P::pos(d, cur ^ 1) + rd.base;
    typename P::vel_t* vel = P::vel(d) + rd.base;
    typename P::vel_t* velt = P::velt(d) + rd.base;
    int32_t* cellid = d.cellid + rd.base;
    int32_t* rank = d.rank + rd.base;
    int32_t* perm = d.perm + rd.base;
    for (int c = tid; c < ncc; c += nt) cnt[c] = 0;
    __syncthreads();
    for (int i = tid; i < rd.N; i += nt) {
        const typename P::pos_t p = pos[i];
        const int c = (P::cellc(p.x, rd) * nc + P::cellc(p.y, rd)) * nc + P::cellc(p.z, rd);
        cellid[i] = c;
        rank[i] = atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    // exclusive scan of the counts: contiguous chunks per thread, then a scan
    // of the chunk sums
    const int chunk = (ncc + nt - 1) / nt;
    const int c0 = tid * chunk, c1 = min(ncc, c0 + chunk);
    int s = 0;
    for (int c = c0; c < c1; ++c) s += cnt[c];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int c = c0; c < c1; ++c) {
        const int n = cnt[c];
        cnt[c] = run;
        run += n;
    }
    __syncthreads();
    if (tid == 0) cnt[ncc] = rd.N;
    __syncthreads();
    int32_t* cstart = d.cell_start + rd.cell_base;
    for (int c = tid; c <= ncc; c += nt) cstart[c] = cnt[c];
    for (int i = tid; i < rd.N; i += nt) perm[cnt[cellid[i]] + rank[i]] = i;
    __syncthreads();
    // order every cell by atom id.  First the ids in cell order (into the
    // free `cellid` scratch), then one wavefront per cell: an atom's place is
    // the number of atoms of its cell with a smaller id, counted through lane
    // shuffles 64 at a time; the next cell's ids are loaded while the
    // current one is ranked.  The ordered slots go to `rank`.
    for (int k = tid; k < rd.N; k += nt) cellid[k] = P::id(pos[perm[k]]);
    __syncthreads();
    {
        const int lane = tid & 63, nw = nt >> 6;
        int c = tid >> 6;
        int a = 0, n = 0, id = 0x7fffffff, mine = 0;
        if (c < ncc) {
            a = cnt[c];
            n = cnt[c + 1] - a;
            id = lane < n ? cellid[a + lane] : 0x7fffffff;
            mine = lane < n ? perm[a + lane] : 0;
        }
        while (c < ncc) {
            const int c2 = c + nw;
            int a2 = 0, n2 = 0, id2 = 0x7fffffff, mine2 = 0;
            if (c2 < ncc) {
                a2 = cnt[c2];
                n2 = cnt[c2 + 1] - a2;
                id2 = lane < n2 ? cellid[a2 + lane] : 0x7fffffff;
                mine2 = lane < n2 ? perm[a2 + lane] : 0;
            }
            if (n <= 64) {
                int rk = 0;
                for (int l = 0; l < n; ++l) rk += __shfl(id, l) < id ? 1 : 0;
                if (lane < n) rank[a + rk] = mine;
            } else {
                for (int bi = 0; bi < n; bi += 64) {
                    const bool vi = bi + lane < n;
                    const int m = vi ? perm[a + bi + lane] : 0;
                    const int myid = vi ? cellid[a + bi + lane] : 0x7fffffff;
                    int rk = 0;
                    for (int bj = 0; bj < n; bj += 64) {
                        const int jid = bj + lane < n ? cellid[a + bj + lane] : 0x7fffffff;
                        for (int l = 0; l < 64; ++l) rk += __shfl(jid, l) < myid ? 1 : 0;
                    }
                    if (vi) rank[a + rk] = m;
                }
            }
            c = c2;
            a = a2;
            n = n2;
            id = id2;
            mine = mine2;
        }
    }
    __syncthreads();
    for (int k = tid; k < rd.N; k += nt) {
        const int src = rank[k];
        tmp[k] = pos[src];
        velt[k] = vel[src];
    }
    __syncthreads();
    typename P::pos_t* xref = P::xref(d) + rd.base;
    for (int k = tid; k < rd.N; k += nt) {
        const typename P::pos_t p = tmp[k];
        pos[k] = p;
        xref[k] = p;
        vel[k] = velt[k];
    }
    if (tid == 0) d.rebuilds[r] += 1;
}

// ---------------------------------------------------------------------------
// Cell-cooperative Verlet list build.  One workgroup per cell: the atoms of
// the 27 neighbouring cells (every cell when there are fewer than 3 per side)
// are staged in LDS, and each i-atom of the cell is tested against them by a
// group of G lanes.  Pass 1 counts each lane's hits, a shuffle scan inside
// the group gives each lane its first list entry, pass 2 writes the entries.
// Entry k of atom i lives at nl[nl_base + ((k / tpa) Np + i) tpa + k % tpa].
template <class P>
struct ListLds {
    static constexpr int CH = P::kF64 ? 1024 : 2048;  // staged candidates per chunk
    typename P::pos_t pos[CH];
    int slot[CH];
    int nb_start[28], nb_pre[28];
    int nnb, total;
};

template <class P>
__device__ void list_cell(const DevState& d, const RepDev& rd, const typename P::pos_t* pos, int c, int tpa,
                          int M, ListLds<P>& sh)
{
    using real = typename P::real;
    constexpr int CH = ListLds<P>::CH;
    const int t = threadIdx.x, nt = blockDim.x;
    const int nc = rd.ncell;
    const int32_t* cstart = d.cell_start + rd.cell_base;
    if (t == 0) {
        int nnb = 0, tot = 0;
        const int cz = c % nc, cy = (c / nc) % nc, cx = c / (nc * nc);
        const int span = nc >= 3 ? 3 : nc;
        for (int ox = 0; ox < span; ++ox)
            for (int oy = 0; oy < span; ++oy)
                for (int oz = 0; oz < span; ++oz) {
                    const int x = nc >= 3 ? (cx + ox - 1 + nc) % nc : ox;
                    const int y = nc >= 3 ? (cy + oy - 1 + nc) % nc : oy;
                    const int z = nc >= 3 ? (cz + oz - 1 + nc) % nc : oz;
                    const int q = (x * nc + y) * nc + z;
                    sh.nb_start[nnb] = cstart[q];
                    sh.nb_pre[nnb] = tot;
                    tot += cstart[q + 1] - cstart[q];
                    ++nnb;
                }
        sh.nb_pre[nnb] = tot;
        sh.nnb = nnb;
        sh.total = tot;
    }
    __syncthreads();
    const int total = sh.total;
    const int ai = cstart[c], ni = cstart[c + 1] - ai;
    const real rl2 = P::rl2(rd);
    const size_t Np = (size_t)rd.Np;
    uint32_t* nl = d.nl + rd.nl_base;
    const int nchunk = (total + CH - 1) / CH;
    auto stage = [&](int c0) {
        const int n = min(CH, total - c0);
        for (int k = t; k < n; k += nt) {
            const int g = c0 + k;
            int b = 0;
            while (sh.nb_pre[b + 1] <= g) ++b;
            const int sl = sh.nb_start[b] + (g - sh.nb_pre[b]);
            sh.pos[k] = pos[sl];
            sh.slot[k] = sl;
        }
    };
    for (int i0 = 0; i0 < ni; i0 += nt) {
        const int nic = min(nt, ni - i0);
        int G = 1;
        while (G < 64 && 2 * G * nic <= nt) G <<= 1;
        const int il = t / G, q = t % G;
        const bool act = il < nic;
        const int islot = ai + i0 + (act ? il : 0);
        const typename P::pos_t pi = pos[islot];
        int cnt = 0;
        for (int ch = 0; ch < nchunk; ++ch) {
            if (nchunk > 1 || i0 == 0) {
                __syncthreads();
                stage(ch * CH);
                __syncthreads();
            }
            const int n = min(CH, total - ch * CH);
            if (act)
                for (int k = q; k < n; k += G) {
                    real dx, dy, dz;
                    P::diff(pi, sh.pos[k], rd, dx, dy, dz);
                    cnt += (dx * dx + dy * dy + dz * dz < rl2 && sh.slot[k] != islot) ? 1 : 0;
                }
        }
        // exclusive scan of the counts inside the group of G lanes
        int off = cnt;
        for (int m = 1; m < G; m <<= 1) {
            const int v = __shfl_up(off, m, G);
            if (q >= m) off += v;
        }
        const int tot_i = __shfl(off, G - 1, G);
        off -= cnt;
        for (int ch = 0; ch < nchunk; ++ch) {
            if (nchunk > 1) {
                __syncthreads();
                stage(ch * CH);
                __syncthreads();
            }
            const int n = min(CH, total - ch * CH);
            if (act)
                for (int k = q; k < n; k += G) {
                    real dx, dy, dz;
                    P::diff(pi, sh.pos[k], rd, dx, dy, dz);
                    if (dx * dx + dy * dy + dz * dz < rl2 && sh.slot[k] != islot) {
                        if (off < M) nl[((size_t)(off / tpa) * Np + islot) * tpa + (off % tpa)] = (uint32_t)sh.slot[k];
                        ++off;
                    }
                }
        }
        if (act && q == 0) {
            d.nn[rd.base + islot] = tot_i < M ? tot_i : M;
            if (tot_i > M) atomicOr(d.overflow, 1u);
        }
    }
    __syncthreads();
}

// Lockstep wrapper: blockIdx.y = replica (from r0), blockIdx.x strides over
// the replica's cells.
template <class P>
__global__ __launch_bounds__(256) void k_listcell(DevState d, StepArgs sa)
{
    const int r = sa.r0 + blockIdx.y;
    if (!sa.force_all && d.flag[(size_t)sa.par * sa.R + r] == 0) return;
    const RepDev rd = d.rep[r];
    __shared__ ListLds<P> sh;
    const typename P::pos_t* pos = P::pos(d, sa.cur) + rd.base;
    const int ncc = rd.ncell * rd.ncell * rd.ncell;
    for (int c = blockIdx.x; c < ncc; c += gridDim.x) list_cell<P>(d, rd, pos, c, sa.tpa, sa.M, sh);
}

// ---------------------------------------------------------------------------
// LJ force (+ energy) over the Verlet list, TPA lanes per atom, then the
// step epilogue selected by MODE:
//   kFused:      v += h F (ends this step), v += h F, x += h v, O, x += h v
//                (the next step's first half; positions to the other buffer)
//   kStop/kStopEnergy: v += h F; store F (and the per-atom energy)
//   kQuery:      F and energy to the query buffer in atom-id order only
//   kRefresh:    store F and the per-atom energy; velocities untouched.
// u(r) = 4 (r^-12 - r^-6) - u(r_c), F_i = 24 (2 r^-14 - r^-8) r_ij for r < r_c
// (Example section: cutoff 2.5; energy shifted, force truncated).
template <class P, int MODE, int TPA>
__global__ __launch_bounds__(256) void k_force(DevState d, StepArgs sa)
{
    using real = typename P::real;
    constexpr bool kEnergy = (MODE == kStopEnergy || MODE == kQuery || MODE == kRefresh);
    const int cur = sa.cur, par = sa.par, R = sa.R;
    const int64_t step_next = sa.step;
    const int b = sa.blk_off + blockIdx.x;
    const int r = sa.tab.rep[b];
    if (r < 0) return;
    const RepDev rd = d.rep[r];
    const int a0 = sa.tab.a0[b];
    if (MODE != kQuery && a0 == 0 && threadIdx.x == 0) d.flag[(size_t)par * R + r] = 0u;  // list consumed
    const int ia = a0 + (int)(threadIdx.x / TPA);
    const int q = (int)(threadIdx.x % TPA);
    const bool valid = ia < rd.N;
    const typename P::pos_t* pos = P::pos(d, cur) + rd.base;
    real fx = 0, fy = 0, fz = 0, e = 0;
    typename P::pos_t pi{};
    if (valid) {
        pi = pos[ia];
        const int nnb = d.nn[rd.base + ia];
        const uint32_t* __restrict__ nlp = d.nl + rd.nl_base + (size_t)ia * TPA + q;
        const size_t stride = (size_t)rd.Np * TPA;
        const int nrow = (nnb - q + TPA - 1) / TPA;
        if constexpr (P::kF64) {
            const double rc2 = rd.rc2d;
            for (int kk = 0; kk < nrow; ++kk) {
                const uint32_t j = nlp[(size_t)kk * stride];
                double dx, dy, dz;
                P::diff(pi, pos[j], rd, dx, dy, dz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2) {
                    const double ir2 = 1.0 / r2;
                    const double ir6 = ir2 * ir2 * ir2;
                    const double ff = 24.0 * ir2 * ir6 * (2.0 * ir6 - 1.0);
                    fx += ff * dx;
                    fy += ff * dy;
                    fz += ff * dz;
                    if constexpr (kEnergy) e += 4.0 * ir6 * (ir6 - 1.0) - sa.ushiftd;
                }
            }
        } else {
            const float rc2 = rd.rc2f, lo = rd.near_lo, hi = rd.near_hi, is2 = rd.inv_s2f;
            const float ushift = (float)sa.ushiftd;
            const uint64_t thr = rd.rc2_exact;
            for (int kk = 0; kk < nrow; ++kk) {
                const uint32_t j = nlp[(size_t)kk * stride];
                const int4 pj = pos[j];
                const int ix = PMixed::wrapdiff(pi.x, pj.x);
                const int iy = PMixed::wrapdiff(pi.y, pj.y);
                const int iz = PMixed::wrapdiff(pi.z, pj.z);
                const float dx = (float)ix, dy = (float)iy, dz = (float)iz;
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                bool in = r2 < rc2;
                if (__builtin_expect(r2 > lo && r2 < hi, 0)) {
                    // within 2^-20 of the cutoff: decide on the exact integer square
                    const uint64_t e2 = (uint64_t)((int64_t)ix * ix) + (uint64_t)((int64_t)iy * iy) +
                                        (uint64_t)((int64_t)iz * iz);
                    in = e2 < thr;
                }
                const float ir2 = __builtin_amdgcn_rcpf(r2) * is2;
                const float ir6 = ir2 * ir2 * ir2;
                const float ff = in ? ir2 * ir6 * __builtin_fmaf(48.0f, ir6, -24.0f) : 0.0f;
                fx = __builtin_fmaf(ff, dx, fx);
                fy = __builtin_fmaf(ff, dy, fy);
                fz = __builtin_fmaf(ff, dz, fz);
                if constexpr (kEnergy) e += in ? __builtin_fmaf(4.0f * ir6, ir6, -4.0f * ir6) - ushift : 0.0f;
            }
        }
    }
#pragma unroll
    for (int m = 1; m < TPA; m <<= 1) {
        fx += __shfl_xor(fx, m, TPA);
        fy += __shfl_xor(fy, m, TPA);
        fz += __shfl_xor(fz, m, TPA);
        if constexpr (kEnergy) e += __shfl_xor(e, m, TPA);
    }
    if (!valid || q != 0) return;
    if constexpr (!P::kF64) {  // grid units -> LJ units
        fx *= rd.sf;
        fy *= rd.sf;
        fz *= rd.sf;
    }
    const int g = rd.base + ia;
    if constexpr (MODE == kQuery) {
        double* o = d.fq + 4 * (size_t)(rd.base + P::id(pi));
        o[0] = (double)fx;
        o[1] = (double)fy;
        o[2] = (double)fz;
        o[3] = (double)e;
        return;
    } else {
        const real hh = MODE == kRefresh ? (real)0 : (real)sa.h;
        typename P::vel_t v = P::vel(d)[g];
        real vx = v.x + hh * fx, vy = v.y + hh * fy, vz = v.z + hh * fz;
        if constexpr (MODE == kFused) {
            const real c1 = (real)sa.c1;
            const real c2 = (real)d.c2[r];
            vx += hh * fx;
            vy += hh * fy;
            vz += hh * fz;
            typename P::pos_t x = P::drift(pi, hh * vx, hh * vy, hh * vz, rd);
            const uint4 w = draw(sa.seed, (uint32_t)P::id(pi), (uint32_t)step_next, (uint32_t)r, kPurposeOStep);
            real z0, z1, z2;
            if constexpr (P::kF64) {
                normals3d(w, z0, z1, z2);
            } else {
                normals3f(w, z0, z1, z2);
            }
            vx = c1 * vx + c2 * z0;
            vy = c1 * vy + c2 * z1;
            vz = c1 * vz + c2 * z2;
            x = P::drift(x, hh * vx, hh * vy, hh * vz, rd);
            P::pos(d, cur ^ 1)[g] = x;
            set_xyz<P>(v, vx, vy, vz);
            P::vel(d)[g] = v;
            real dx, dy, dz;
            P::diff(x, P::xref(d)[g], rd, dx, dy, dz);
            if (dx * dx + dy * dy + dz * dz > P::lim2(rd))
                atomicOr(&d.flag[(size_t)(par ^ 1) * R + r], 1u);
        } else {
            set_xyz<P>(v, vx, vy, vz);
            P::vel(d)[g] = v;
            typename P::vel_t f;
            f.x = fx;
            f.y = fy;
            f.z = fz;
            f.w = 0;
            P::frc(d)[g] = f;
            if constexpr (MODE == kStopEnergy || MODE == kRefresh) P::epot(d)[g] = e;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-replica potential energy in FP64: fixed-order strided sums of the
// per-atom energies, then a fixed tree; U = (1/2) sum_i e_i.
template <class P>
__global__ __launch_bounds__(256) void k_energy(DevState d, StepArgs sa)
{
    const int r = sa.r0 + blockIdx.x;
    const RepDev rd = d.rep[r];
    __shared__ double part[256];
    double s = 0.0;
    const typename P::real* e = P::epot(d) + rd.base;
    for (int i = threadIdx.x; i < rd.N; i += 256) s += (double)e[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.U[r] = 0.5 * part[0];
}

// ---------------------------------------------------------------------------
// Exchange attempt k (Implementation section): ladder slots (j, j+1) with
// j = k mod 2 are paired; for the replicas a, b holding them
// D = (1/T_j - 1/T_{j+1}) (U_a - U_b); the 53-bit uniform of the lower
// replica id decides: accept iff D >= 0 or u < exp(D).  Accepted pairs swap
// slots; every replica gets its velocity factor alpha = sqrt(T_new/T_old)
// (1 if not swapped) and the noise amplitude of its new temperature.
__device__ void exchange_body(const double* U, const double* Tl, int32_t* slot, int R, int64_t k, uint64_t seed,
                              double* alpha, double* c2, double c1sq, int64_t* att, int64_t* acc, XRec* log,
                              int64_t* log_count, int64_t log_cap, const int64_t* steps, int64_t step_all,
                              int32_t master, uint8_t* dec)
{
    __shared__ int rep[4096];
    __shared__ int64_t lbase;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int r = tid; r < R; r += nt) {
        rep[slot[r]] = r;
        if (alpha) alpha[r] = 1.0;
    }
    if (tid == 0) lbase = log_count ? *log_count : 0;
    __syncthreads();
    const int j0 = (int)(k & 1);
    const int npairs = (R - j0) / 2;
    for (int p = tid; p < npairs; p += nt) {
        const int j = j0 + 2 * p;
        const int a = rep[j], b = rep[j + 1];
        const double Ta = Tl[j], Tb = Tl[j + 1];
        const double delta = (1.0 / Ta - 1.0 / Tb) * (U[a] - U[b]);
        const double u = uniform53(seed, k, a < b ? a : b);
        const int ok = (delta >= 0.0 || u < exp(delta)) ? 1 : 0;
        if (dec) dec[j] = (uint8_t)ok;
        if (att) att[j] += 1;
        if (acc) acc[j] += ok;
        if (log) {
            XRec rec;
            rec.attempt = k;
            rec.master = master;
            rec.slot_lo = j;
            rec.rep_a = a;
            rec.rep_b = b;
            rec.step_a = step_all >= 0 ? step_all : steps[a];
            rec.step_b = step_all >= 0 ? step_all : steps[b];
            rec.U_a = U[a];
            rec.U_b = U[b];
            rec.T_a = Ta;
            rec.T_b = Tb;
            rec.u = u;
            rec.accepted = ok;
            rec.pad_ = 0;
            log[(lbase + p) % log_cap] = rec;
        }
        if (ok) {
            slot[a] = j + 1;
            slot[b] = j;
            if (alpha) {
                alpha[a] = sqrt(Tb / Ta);
                alpha[b] = sqrt(Ta / Tb);
            }
            if (c2) {
                c2[a] = sqrt((1.0 - c1sq) * Tb);
                c2[b] = sqrt((1.0 - c1sq) * Ta);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && log_count) *log_count = lbase + npairs;
}

__global__ __launch_bounds__(1024) void k_exchange(DevState d, int R, int64_t k, uint64_t seed, double c1sq,
                                                   int32_t master, int64_t log_cap, int64_t step_all)
{
    exchange_body(d.U, d.Tl, d.slot, R, k, seed, d.alpha, d.c2, c1sq, d.attempts, d.accepts, d.log, d.log_count,
                  log_cap, d.steps, step_all, master, nullptr);
}

__global__ __launch_bounds__(1024) void k_test_exchange(const double* U, const double* Tl, int32_t* slot, int R,
                                                        uint64_t seed, int64_t k, uint8_t* dec)
{
    for (int j = threadIdx.x; j < R - 1; j += blockDim.x) dec[j] = 255;
    __syncthreads();
    exchange_body(U, Tl, slot, R, k, seed, nullptr, nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, 1, nullptr, 0,
                  -1, dec);
}

__global__ void k_test_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int n, uint32_t* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 w = philox10(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]), k0, k1);
    out[4 * i] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
}

__global__ void k_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 w = draw(seed, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    if (fp64) {
        double z0, z1, z2;
        normals3d(w, z0, z1, z2);
        out[3 * i] = z0;
        out[3 * i + 1] = z1;
        out[3 * i + 2] = z2;
    } else {
        float z0, z1, z2;
        normals3f(w, z0, z1, z2);
        out[3 * i] = z0;
        out[3 * i + 1] = z1;
        out[3 * i + 2] = z2;
    }
}

__global__ void k_clear_flags(DevState d, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d.flag[i] = 0u;
}

__global__ void k_set_steps(DevState d, int R, int64_t step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R) d.steps[i] = step;
}

// ---------------------------------------------------------------------------
// Launch wrappers.
template <class P>
static hipError_t start_t(const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL(k_start<P>, dim3(nblk), dim3(sa.block), 0, st, d, sa);
    return hipGetLastError();
}

hipError_t launch_start(bool fp64, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    return fp64 ? start_t<PF64>(d, sa, nblk, st) : start_t<PMixed>(d, sa, nblk, st);
}

hipError_t launch_reorder(bool fp64, const DevState& d, const StepArgs& sa, int nrep, hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_reorder<PF64>, dim3(nrep), dim3(kReorderThreads), 0, st, d, sa);
    else
        hipLaunchKernelGGL(k_reorder<PMixed>, dim3(nrep), dim3(kReorderThreads), 0, st, d, sa);
    return hipGetLastError();
}

hipError_t launch_listbuild(bool fp64, const DevState& d, const StepArgs& sa, int nrep, int cells_max, hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    const dim3 grid(cells_max < 64 ? cells_max : 64, nrep);
    if (fp64)
        hipLaunchKernelGGL(k_listcell<PF64>, grid, dim3(256), 0, st, d, sa);
    else
        hipLaunchKernelGGL(k_listcell<PMixed>, grid, dim3(256), 0, st, d, sa);
    return hipGetLastError();
}

template <class P, int MODE>
static hipError_t force_mode(const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    switch (sa.tpa) {
    case 1: hipLaunchKernelGGL((k_force<P, MODE, 1>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    case 2: hipLaunchKernelGGL((k_force<P, MODE, 2>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    case 4: hipLaunchKernelGGL((k_force<P, MODE, 4>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    case 8: hipLaunchKernelGGL((k_force<P, MODE, 8>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class P>
static hipError_t force_t(StepMode mode, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    switch (mode) {
    case kFused: return force_mode<P, kFused>(d, sa, nblk, st);
    case kStop: return force_mode<P, kStop>(d, sa, nblk, st);
    case kStopEnergy: return force_mode<P, kStopEnergy>(d, sa, nblk, st);
    case kQuery: return force_mode<P, kQuery>(d, sa, nblk, st);
    case kRefresh: return force_mode<P, kRefresh>(d, sa, nblk, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_force(bool fp64, StepMode mode, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    return fp64 ? force_t<PF64>(mode, d, sa, nblk, st) : force_t<PMixed>(mode, d, sa, nblk, st);
}

hipError_t launch_energy(bool fp64, const DevState& d, const StepArgs& sa, int nrep, hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_energy<PF64>, dim3(nrep), dim3(256), 0, st, d, sa);
    else
        hipLaunchKernelGGL(k_energy<PMixed>, dim3(nrep), dim3(256), 0, st, d, sa);
    return hipGetLastError();
}

hipError_t launch_exchange(const DevState& d, int R, int64_t attempt, uint64_t seed, double c1sq, int32_t master,
                           int64_t log_cap, int64_t step_all, hipStream_t st)
{
    hipLaunchKernelGGL(k_exchange, dim3(1), dim3(1024), 0, st, d, R, attempt, seed, c1sq, master, log_cap, step_all);
    return hipGetLastError();
}

hipError_t launch_clear_flags(const DevState& d, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_flags, dim3((n + 255) / 256), dim3(256), 0, st, d, n);
    return hipGetLastError();
}

hipError_t launch_set_steps(const DevState& d, int R, int64_t step, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_steps, dim3((R + 255) / 256), dim3(256), 0, st, d, R, step);
    return hipGetLastError();
}

hipError_t launch_test_exchange(const double* U, const double* Tl, int32_t* slot, int R, uint64_t seed,
                                int64_t attempt, uint8_t* dec, hipStream_t st)
{
    hipLaunchKernelGGL(k_test_exchange, dim3(1), dim3(1024), 0, st, U, Tl, slot, R, seed, attempt, dec);
    return hipGetLastError();
}

hipError_t launch_test_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, int n, uint32_t* out,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_test_philox, dim3((n + 255) / 256), dim3(256), 0, st, ctr, key0, key1, n, out);
    return hipGetLastError();
}

hipError_t launch_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_test_normals, dim3((n + 255) / 256), dim3(256), 0, st, fp64, seed, ctr, n, out);
    return hipGetLastError();
}

}  // namespace re
