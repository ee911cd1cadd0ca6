// re_kernels.hip -- lockstep kernels of the replica-exchange LJ engine:
// one launch per phase for a batch of replicas (the batched lockstep form)
// or for one replica (the plain per-replica form), plus the exchange kernel
// and the test hooks.  The per-atom arithmetic lives in re_device.hpp.
#include "re_device.hpp"
#include "../../include/re.h"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace re {

template <class P>
__global__ __launch_bounds__(256) void k_start(DevState d, StepArgs sa)
{
    const int b = sa.blk_off + blockIdx.x;
    const int r = sa.tab.rep[b];
    if (r < 0) return;
    const RepDev rd = d.rep[r];
    const int i = sa.tab.a0[b] + threadIdx.x;
    if (i >= rd.N) return;
    start_atom<P>(d, sa, rd, r, i, sa.cur, sa.step, sa.apply_alpha != 0);
}

// ---------------------------------------------------------------------------
// List updates.  A work table first lists the replicas whose update flag is
// set, with prefix sums of their list-build blocks, atoms and cell entries;
// the reorder and list kernels then run over those replicas' work only.

constexpr int kListAPB = 256 / kListLanes;  // atoms per list-build block

// Last k in [0, n) with pre[k] <= v (pre nondecreasing, pre[0] = 0 <= v).
__device__ __forceinline__ int work_slot(const int32_t* pre, int n, int v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Table layout (nrep replicas from sa.r0): blk[nrep+1], atm[nrep+1],
// cel[nrep+1] prefix sums; rep[nrep] the rebuilt replicas in order; nflag.
struct WorkTable {
    int32_t *blk, *atm, *cel, *rep, *nflag;
};
__device__ __forceinline__ WorkTable work_table(const DevState& d, int nrep)
{
    WorkTable w;
    w.blk = d.wtab;
    w.atm = w.blk + nrep + 1;
    w.cel = w.atm + nrep + 1;
    w.rep = w.cel + nrep + 1;
    w.nflag = w.rep + nrep;
    return w;
}

__device__ __forceinline__ void rebuild_work(const DevState& d, const StepArgs& sa, int k, int& nb, int& na, int& nc,
                                             int& nf)
{
    const int r = sa.r0 + k;
    const bool f = sa.force_all || d.flag[(size_t)sa.par * sa.R + r] == rebuild_tag(sa.step);
    const int N = d.rep[r].N, c = d.rep[r].ncell;
    nb = f ? (N + kListAPB - 1) / kListAPB : 0;
    na = f ? N : 0;
    nc = f ? c * c * c + 1 : 0;
    nf = f ? 1 : 0;
}

// One workgroup of 1024: each thread sums a chunk of replicas, a two-level
// shuffle scan gives the chunk offsets, the chunk writes its prefixes.
__global__ __launch_bounds__(1024) void k_rebuild_table(DevState d, StepArgs sa, int nrep)
{
    __shared__ int wsum[4][16];
    __shared__ int wpre[4][16];
    const WorkTable w = work_table(d, nrep);
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    const int chunk = (nrep + nt - 1) / nt;
    const int k0 = min(nrep, tid * chunk), k1 = min(nrep, k0 + chunk);
    int s[4] = {0, 0, 0, 0};
    for (int k = k0; k < k1; ++k) {
        int v[4];
        rebuild_work(d, sa, k, v[0], v[1], v[2], v[3]);
        for (int q = 0; q < 4; ++q) s[q] += v[q];
    }
    int x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        x[q] = s[q];
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x[q], o, 64);
            if (lane >= o) x[q] += y;
        }
        if (lane == 63) wsum[q][wv] = x[q];
    }
    __syncthreads();
    if (tid < 4) {
        int run = 0;
        for (int u = 0; u < nw; ++u) {
            wpre[tid][u] = run;
            run += wsum[tid][u];
        }
    }
    __syncthreads();
    int run[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) run[q] = wpre[q][wv] + x[q] - s[q];
    for (int k = k0; k < k1; ++k) {
        int v[4];
        rebuild_work(d, sa, k, v[0], v[1], v[2], v[3]);
        w.blk[k] = run[0];
        w.atm[k] = run[1];
        w.cel[k] = run[2];
        if (v[3]) w.rep[run[3]] = sa.r0 + k;
        for (int q = 0; q < 4; ++q) run[q] += v[q];
    }
    if (tid == nt - 1) {
        w.blk[nrep] = run[0];
        w.atm[nrep] = run[1];
        w.cel[nrep] = run[2];
        *w.nflag = run[3];
    }
}

// Reorder with one workgroup per rebuilt replica.
template <class P>
__global__ __launch_bounds__(kReorderThreads) void k_reorder(DevState d, StepArgs sa, int nrep)
{
    __shared__ int cnt[kMaxCells + 1];
    __shared__ int part[kReorderThreads];
    const WorkTable w = work_table(d, nrep);
    for (int j = blockIdx.x; j < *w.nflag; j += gridDim.x) {
        const int r = w.rep[j];
        const RepDev rd = d.rep[r];
        reorder_replica<P>(d, rd, r, sa.cur, cnt, part);
    }
}

// Reorder with grid-wide passes over the rebuilt replicas' atoms, the same
// result as reorder_replica: counting sort into the cell grid (counts in the
// cell-start array), each cell ordered by atom id, positions and velocities
// gathered into the new order, x_ref := x.
#define RE_FOR_WORK(pre, ...)                                                                \
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < (pre)[nrep];                    \
         g += gridDim.x * blockDim.x) {                                                      \
        const int k = work_slot((pre), nrep, g);                                             \
        const int r = sa.r0 + k;                                                             \
        const RepDev rd = d.rep[r];                                                          \
        const int i = g - (pre)[k];                                                          \
        (void)r;                                                                             \
        __VA_ARGS__                                                                          \
    }

template <class P>
__global__ __launch_bounds__(256) void k_ro_zero(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.cel, { d.cell_start[rd.cell_base + i] = 0; })
}

template <class P>
__global__ __launch_bounds__(256) void k_ro_count(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.atm, {
        const int nc = rd.ncell;
        const typename P::pos_t p = P::pos(d, sa.cur)[rd.base + i];
        const int c = (P::cellc(p.x, rd) * nc + P::cellc(p.y, rd)) * nc + P::cellc(p.z, rd);
        d.cellid[rd.base + i] = c;
        d.rank[rd.base + i] = atomicAdd(&d.cell_start[rd.cell_base + c], 1);
    })
}

// exclusive scan of each rebuilt replica's counts in place (one workgroup of
// 1024 per replica); the entry past the last cell becomes N
__global__ __launch_bounds__(1024) void k_ro_scan(DevState d, StepArgs sa, int nrep)
{
    __shared__ int wsum[16];
    const WorkTable w = work_table(d, nrep);
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    for (int j = blockIdx.x; j < *w.nflag; j += gridDim.x) {
        const RepDev rd = d.rep[w.rep[j]];
        const int ncc = rd.ncell * rd.ncell * rd.ncell;
        int32_t* cs = d.cell_start + rd.cell_base;
        const int chunk = (ncc + nt - 1) / nt;
        const int c0 = min(ncc, tid * chunk), c1 = min(ncc, c0 + chunk);
        int s = 0;
        for (int c = c0; c < c1; ++c) s += cs[c];
        int x = s;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int base = 0;
        for (int u = 0; u < wv; ++u) base += wsum[u];
        int run = base + x - s;
        for (int c = c0; c < c1; ++c) {
            const int n = cs[c];
            cs[c] = run;
            run += n;
        }
        if (tid == 0) cs[ncc] = rd.N;
        (void)nw;
        __syncthreads();
    }
}

template <class P>
__global__ __launch_bounds__(256) void k_ro_scatter(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.atm, {
        const int32_t* cs = d.cell_start + rd.cell_base;
        d.perm[rd.base + cs[d.cellid[rd.base + i]] + d.rank[rd.base + i]] = i;
    })
}

template <class P>
__global__ __launch_bounds__(256) void k_ro_ids(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.atm, { d.cellid[rd.base + i] = P::id(P::pos(d, sa.cur)[rd.base + d.perm[rd.base + i]]); })
}

template <class P>
__global__ __launch_bounds__(256) void k_ro_rank(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.atm, {
        const int ncc = rd.ncell * rd.ncell * rd.ncell;
        const int32_t* cs = d.cell_start + rd.cell_base;
        const int32_t* ids = d.cellid + rd.base;
        int lo = 0, hi = ncc - 1;  // the cell of sorted slot i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cs[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int a = cs[lo], e = cs[lo + 1];
        const int myid = ids[i];
        int rk = 0;
        for (int m = a; m < e; ++m) rk += ids[m] < myid ? 1 : 0;
        d.rank[rd.base + a + rk] = d.perm[rd.base + i];
    })
}

template <class P>
__global__ __launch_bounds__(256) void k_ro_gather(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.atm, {
        const int src = d.rank[rd.base + i];
        P::pos(d, sa.cur ^ 1)[rd.base + i] = P::pos(d, sa.cur)[rd.base + src];
        P::velt(d)[rd.base + i] = P::vel(d)[rd.base + src];
    })
}

template <class P>
__global__ __launch_bounds__(256) void k_ro_copy(DevState d, StepArgs sa, int nrep)
{
    const WorkTable w = work_table(d, nrep);
    RE_FOR_WORK(w.atm, {
        const typename P::pos_t p = P::pos(d, sa.cur ^ 1)[rd.base + i];
        P::pos(d, sa.cur)[rd.base + i] = p;
        P::xref(d)[rd.base + i] = p;
        P::vel(d)[rd.base + i] = P::velt(d)[rd.base + i];
        if (i == 0) d.rebuilds[r] += 1;
    })
}
#undef RE_FOR_WORK

// List build over the rebuilt replicas' atoms: block vb of the table holds
// kListAPB atoms of one replica.
template <class P>
__global__ __launch_bounds__(256) void k_listrows(DevState d, StepArgs sa, int nrep)
{
    constexpr int W = list_lds_words<kListLanes>();
    __shared__ int lds[256 * W];
    const WorkTable w = work_table(d, nrep);
    for (int vb = blockIdx.x; vb < w.blk[nrep]; vb += gridDim.x) {
        const int k = work_slot(w.blk, nrep, vb);
        const int r = sa.r0 + k;
        const RepDev rd = d.rep[r];
        const int i = (vb - w.blk[k]) * kListAPB + (int)(threadIdx.x / kListLanes);
        const typename P::pos_t* pos = P::pos(d, sa.cur) + rd.base;
        list_rows<P, kListLanes>(d, rd, pos, pos, d.cell_start + rd.cell_base, i, i < rd.N, (int)(threadIdx.x % kListLanes),
                                 rd.tpa, sa.M, lds + threadIdx.x * W);
    }
}

// Force + epilogue of one block of TPA-lane atom groups.  With TPA > 1 the
// sums go through LDS and the step epilogues (noise, integration) then run
// one atom per thread in the block's first blockDim/TPA threads, instead of
// on one lane of each group while the others idle.
template <class P, int MODE, int TPA>
__device__ __forceinline__ void force_block(const DevState& d, const StepArgs& sa, const RepDev& rd, int r, int a0)
{
    const int tid = (int)threadIdx.x;
    const int ia = a0 + tid / TPA;
    if constexpr (TPA == 1) {
        force_atom<P, MODE, TPA>(d, sa, rd, r, ia, 0, ia < rd.N, sa.cur, sa.step, sa.par);
    } else {
        using real = typename P::real;
        using real4 = typename P::vel_t;
        __shared__ real4 lf[256 / TPA];
        __shared__ typename P::pos_t lp[256 / TPA];
        typename P::pos_t pi;
        real fx, fy, fz, e;
        force_sum<P, MODE, TPA>(d, sa, rd, P::pos(d, sa.cur) + rd.base, ia, tid % TPA, ia < rd.N, pi, fx, fy, fz, e);
        // this thread's epilogue atom; its velocity and x_ref are loaded
        // before the barrier so that their latency overlaps it
        const int ja = a0 + tid;
        const bool epi = tid < (int)blockDim.x / TPA && ja < rd.N;
        real4 v0{};
        typename P::pos_t xr0{};
        if (epi) {
            if constexpr (MODE != kQuery) v0 = P::vel(d)[rd.base + ja];
            if constexpr (MODE == kFused) xr0 = P::xref(d)[rd.base + ja];
        }
        if (tid % TPA == 0 && ia < rd.N) {
            real4 f;
            f.x = fx;
            f.y = fy;
            f.z = fz;
            f.w = e;
            lf[tid / TPA] = f;
            lp[tid / TPA] = pi;
        }
        __syncthreads();
        if (epi) {
            const real4 f = lf[tid];
            force_epilogue_v<P, MODE>(d, sa, rd, r, ja, sa.cur, sa.step, sa.par, lp[tid], f.x, f.y, f.z, f.w, v0, xr0);
        }
    }
}

// Force + epilogue; the first block of each replica also marks the pending
// velocity factor applied.  TPA = 0: each block takes the lanes per atom of
// its replica (a block table built with blockDim/tpa atoms per block).
template <class P, int MODE, int TPA>
__global__ __launch_bounds__(256) void k_force(DevState d, StepArgs sa)
{
    const int b = sa.blk_off + blockIdx.x;
    const int r = sa.tab.rep[b];
    if (r < 0) return;
    const RepDev rd = d.rep[r];
    const int a0 = sa.tab.a0[b];
    if (MODE != kQuery && a0 == 0 && threadIdx.x == 0) d.alpha[r] = 1.0;
    if constexpr (TPA != 0) {
        force_block<P, MODE, TPA>(d, sa, rd, r, a0);
    } else {
        switch (rd.tpa) {
        case 1: force_block<P, MODE, 1>(d, sa, rd, r, a0); break;
        case 2: force_block<P, MODE, 2>(d, sa, rd, r, a0); break;
        case 4: force_block<P, MODE, 4>(d, sa, rd, r, a0); break;
        default: force_block<P, MODE, 8>(d, sa, rd, r, a0); break;
        }
    }
}

// Per-replica reductions at a stopped boundary: the potential energy
// (do_u) and the velocity rescale factor of the thermostat (do_svr).
template <class P>
__global__ __launch_bounds__(256) void k_energy(DevState d, StepArgs sa)
{
    __shared__ double part[kRedLds];
    const int r = sa.r0 + blockIdx.x;
    const RepDev rd = d.rep[r];
    if (sa.do_u) energy_replica<P>(d, rd, r, part);
    if (sa.do_svr) svr_replica<P>(d, rd, r, sa.step, sa.seed, sa.svr_c, false, 0.0, part);
}

// ---------------------------------------------------------------------------
// Exchange attempt k (Implementation section): ladder slots (j, j+1) with
// j = k mod 2 are paired -- or, with non-nearest-neighbour exchanges, slots
// (j, j+d) at the attempt's distance d (j >= o = (k mod 2) d with
// floor((j - o)/d) even); for the replicas a, b holding them
// D = (1/T_j - 1/T_{j+1}) (U_a - U_b); the 53-bit uniform of the lower
// replica id decides: accept iff D >= 0 or u < exp(D).  Accepted pairs swap
// slots; each swapped replica's pending velocity factor is multiplied by
// sqrt(T_new/T_old) and it takes the noise amplitude of its new temperature.
__device__ void exchange_body(const double* U, const double* Tl, int32_t* slot, int R, int64_t k, uint64_t seed,
                              int max_distance, double* alpha, double* c2, double c1sq, int64_t* att, int64_t* acc,
                              XRec* log, int64_t* log_count, int64_t log_cap, const int64_t* steps,
                              int64_t step_all, int32_t master, uint8_t* dec)
{
    __shared__ int rep[4096];
    __shared__ int64_t lbase;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int r = tid; r < R; r += nt) rep[slot[r]] = r;
    if (tid == 0) lbase = log_count ? *log_count : 0;
    __syncthreads();
    // pairs (j, j + dk): j >= o with floor((j - o) / dk) even; the p-th
    // such j is o + 2 dk (p / dk) + p mod dk
    const int dk = pattern_distance(seed, k, max_distance);
    const int o = (int)(k & 1) * dk;
    const int span = R - dk - o;
    const int npairs = span <= 0 ? 0 : (span / (2 * dk)) * dk + min(span % (2 * dk), dk);
    for (int p = tid; p < npairs; p += nt) {
        const int j = o + 2 * dk * (p / dk) + p % dk, h = j + dk;
        const int a = rep[j], b = rep[h];
        const double Ta = Tl[j], Tb = Tl[h];
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
            rec.slot_hi = h;
            log[(lbase + p) % log_cap] = rec;
        }
        if (ok) {
            slot[a] = h;
            slot[b] = j;
            if (alpha) {  // factors of consecutive exchanges compose
                alpha[a] *= sqrt(Tb / Ta);
                alpha[b] *= sqrt(Ta / Tb);
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
                                                   int32_t master, int64_t log_cap, int64_t step_all, int maxd)
{
    exchange_body(d.U, d.Tl, d.slot, R, k, seed, maxd, d.alpha, d.c2, c1sq, d.attempts, d.accepts, d.log,
                  d.log_count, log_cap, d.steps, step_all, master, nullptr);
}

__global__ __launch_bounds__(1024) void k_test_exchange(const double* U, const double* Tl, int32_t* slot, int R,
                                                        uint64_t seed, int64_t k, int maxd, uint8_t* dec)
{
    for (int j = threadIdx.x; j < R - 1; j += blockDim.x) dec[j] = 255;
    __syncthreads();
    exchange_body(U, Tl, slot, R, k, seed, maxd, nullptr, nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, 1,
                  nullptr, 0, -1, dec);
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

// P: the precision policy of the reorder; PL: that of the list build (its
// entry type)
template <class P, class PL>
static hipError_t rebuild_t(const DevState& d, const StepArgs& sa, int nrep, int64_t atoms, bool wide, hipStream_t st)
{
    hipLaunchKernelGGL(k_rebuild_table, dim3(1), dim3(1024), 0, st, d, sa, nrep);
    const int gatom = (int)std::min<int64_t>((atoms + 255) / 256, 4096);
    if (wide) {
        const int gcell = std::min(4096, nrep * (kMaxCells + 1) / 256 + 1);
        hipLaunchKernelGGL(k_ro_zero<P>, dim3(gcell), dim3(256), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_count<P>, dim3(gatom), dim3(256), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_scan, dim3(std::min(nrep, 1024)), dim3(1024), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_scatter<P>, dim3(gatom), dim3(256), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_ids<P>, dim3(gatom), dim3(256), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_rank<P>, dim3(gatom), dim3(256), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_gather<P>, dim3(gatom), dim3(256), 0, st, d, sa, nrep);
        hipLaunchKernelGGL(k_ro_copy<P>, dim3(gatom), dim3(256), 0, st, d, sa, nrep);
    } else {
        hipLaunchKernelGGL(k_reorder<P>, dim3(std::min(nrep, 1024)), dim3(kReorderThreads), 0, st, d, sa, nrep);
    }
    const int gblk = (int)std::min<int64_t>(atoms / kListAPB + nrep, 8192);
    hipLaunchKernelGGL(k_listrows<PL>, dim3(gblk), dim3(256), 0, st, d, sa, nrep);
    return hipGetLastError();
}

hipError_t launch_rebuild(bool fp64, const DevState& d, const StepArgs& sa, int nrep, int64_t atoms, bool wide,
                          hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    if (fp64) return rebuild_t<PF64, PF64>(d, sa, nrep, atoms, wide, st);
    return sa.n16 ? rebuild_t<PMixed, PMixed16>(d, sa, nrep, atoms, wide, st)
                  : rebuild_t<PMixed, PMixed>(d, sa, nrep, atoms, wide, st);
}

template <class P, int MODE>
static hipError_t force_mode(const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    switch (sa.tpa) {
    case 0: hipLaunchKernelGGL((k_force<P, MODE, 0>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
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
    if (fp64) return force_t<PF64>(mode, d, sa, nblk, st);
    return sa.n16 ? force_t<PMixed16>(mode, d, sa, nblk, st) : force_t<PMixed>(mode, d, sa, nblk, st);
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
                           int64_t log_cap, int64_t step_all, int max_distance, hipStream_t st)
{
    hipLaunchKernelGGL(k_exchange, dim3(1), dim3(1024), 0, st, d, R, attempt, seed, c1sq, master, log_cap, step_all,
                       max_distance);
    return hipGetLastError();
}

hipError_t launch_set_steps(const DevState& d, int R, int64_t step, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_steps, dim3((R + 255) / 256), dim3(256), 0, st, d, R, step);
    return hipGetLastError();
}

hipError_t launch_test_exchange(const double* U, const double* Tl, int32_t* slot, int R, uint64_t seed,
                                int64_t attempt, int max_distance, uint8_t* dec, hipStream_t st)
{
    hipLaunchKernelGGL(k_test_exchange, dim3(1), dim3(1024), 0, st, U, Tl, slot, R, seed, attempt, max_distance, dec);
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

// ---------------------------------------------------------------------------
// re_test_exchange without any allocation.  The staging of its inputs
// (energies, ladder, slots) and of its decisions is a file-scope device
// array, one copy per GPU; each device's copy is located once, with that
// device current, and only that address is handed to copies and kernels.
namespace {
constexpr int kStaticMaxR = 4096;  // replicas per call
constexpr size_t kStU = 0, kStT = 8 * (size_t)kStaticMaxR, kStSlot = 16 * (size_t)kStaticMaxR,
                 kStDec = 20 * (size_t)kStaticMaxR, kStBytes = 21 * (size_t)kStaticMaxR;  // 84 KiB
constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
unsigned char* g_static_ptr[kStaticMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStBytes];

extern "C" int re_test_exchange_noalloc(const double* U, const double* T, const int32_t* slot, int R, uint64_t seed,
                                        int64_t attempt, int max_distance, uint8_t* decisions)
{
    if (!U || !T || !slot || !decisions || R < 1 || max_distance < 1)
        return re::fail_noctx(RE_EINVAL, "re_test_exchange_noalloc: bad arguments");
    if (R > kStaticMaxR)
        return re::fail_noctx(RE_EINVAL, "re_test_exchange_noalloc: R = %d exceeds its static staging of %d replicas",
                              R, kStaticMaxR);
    unsigned char seen[kStaticMaxR];
    std::memset(seen, 0, (size_t)R);
    for (int r = 0; r < R; ++r) {
        if (slot[r] < 0 || slot[r] >= R || seen[slot[r]]++)
            return re::fail_noctx(RE_EINVAL, "re_test_exchange_noalloc: slot is not a permutation");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return re::fail_noctx(RE_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kStaticMaxDevices)
        return re::fail_noctx(RE_EDEVICE, "re_test_exchange_noalloc: device index %d out of range", dev);
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!g_static_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return re::fail_noctx(RE_EDEVICE, "hipGetSymbolAddress of the static staging: %s",
                                      hipGetErrorString(e));
            g_static_ptr[dev] = static_cast<unsigned char*>(p);
        }
        base = g_static_ptr[dev];
    }
    double* dU = reinterpret_cast<double*>(base + kStU);
    double* dT = reinterpret_cast<double*>(base + kStT);
    int32_t* ds = reinterpret_cast<int32_t*>(base + kStSlot);
    uint8_t* dd = base + kStDec;
    // every word the kernel reads is written by this call's copies (U, T and
    // slot for the R replicas) or by the kernel itself (decisions), so
    // nothing left by an earlier call is read
    e = hipMemcpy(dU, U, (size_t)R * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dT, T, (size_t)R * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ds, slot, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = re::launch_test_exchange(dU, dT, ds, R, seed, attempt, max_distance, dd, nullptr);
    if (e == hipSuccess && R > 1) e = hipMemcpy(decisions, dd, (size_t)(R - 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return re::fail_noctx(RE_EDEVICE, "re_test_exchange_noalloc: %s", hipGetErrorString(e));
    return RE_OK;
}
