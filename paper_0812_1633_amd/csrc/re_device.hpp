// re_device.hpp -- device code shared by the lockstep kernels
// (re_kernels.hip) and the persistent engine (re_persist.hip).
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
#pragma once
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

// Pairing distance of exchange attempt k: 1 + (w0 mod max_distance), w0 the
// first word of Philox counter (k low, k high, 0, purpose 5); 1 when
// max_distance is 1 (the nearest-neighbour pattern).
__device__ __forceinline__ int pattern_distance(uint64_t seed, int64_t k, int max_distance)
{
    if (max_distance <= 1) return 1;
    const uint4 w = draw(seed, (uint32_t)(uint64_t)k, (uint32_t)((uint64_t)k >> 32), 0u, kPurposePattern);
    return 1 + (int)(w.x % (uint32_t)max_distance);
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
    // neighbour-list entries: the neighbour's byte offset from the replica's
    // first position (32 bits)
    using entry_t = uint32_t;
    static constexpr bool kSlotEntries = false;
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
    // position in cell units, [0, ncell) (FP32: for conservative bounds only)
    __device__ static float cellpos(int x, const RepDev& rd)
    {
        return (float)((uint32_t)x ^ 0x80000000u) * ((float)rd.ncell * 0x1p-32f);
    }
    __device__ static real rc2(const RepDev& rd) { return rd.rc2f; }
    __device__ static real lim2(const RepDev& rd) { return rd.lim2f; }
    // List-build key: the top 16 bits of each coordinate, x and y packed in
    // one word, z alone (a grid of 2^16 points per box side)
    using key_t = uint2;
    __device__ static key_t list_key(const pos_t& p)
    {
        return make_uint2(((uint32_t)p.x >> 16) | ((uint32_t)p.y & 0xffff0000u), (uint32_t)p.z >> 16);
    }
    __device__ static key_t list_key(const key_t& k) { return k; }
    // Within the list radius, on keys: the 16-bit differences wrap (the
    // minimum image on the coarse grid), their squares sum exactly in 32
    // bits, and rd.rl2q bounds that sum for every pair closer than the list
    // radius (each key difference is within one grid step of the true one)
    __device__ static bool list_close(const key_t& a, const key_t& b, const RepDev& rd)
    {
        typedef short short2_t __attribute__((ext_vector_type(2)));
        const short2_t dxy = __builtin_bit_cast(short2_t, a.x) - __builtin_bit_cast(short2_t, b.x);
        const short2_t dz = __builtin_bit_cast(short2_t, a.y) - __builtin_bit_cast(short2_t, b.y);
        const int r2 = __builtin_amdgcn_sdot2(dz, dz, __builtin_amdgcn_sdot2(dxy, dxy, 0, false), false);
        return (uint32_t)r2 < rd.rl2q;
    }
};

struct PF64 {
    using pos_t = double4;
    using vel_t = double4;
    using real = double;
    static constexpr bool kF64 = true;
    using entry_t = uint32_t;  // byte offsets, as in PMixed
    static constexpr bool kSlotEntries = false;
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
    __device__ static float cellpos(double x, const RepDev& rd) { return (float)((x / rd.L + 0.5) * (double)rd.ncell); }
    __device__ static real rc2(const RepDev& rd) { return rd.rc2d; }
    __device__ static real lim2(const RepDev& rd) { return rd.lim2d; }
    // the list build tests FP64 positions directly
    using key_t = pos_t;
    __device__ static const key_t& list_key(const pos_t& p) { return p; }
    __device__ static bool list_close(const key_t& a, const key_t& b, const RepDev& rd)
    {
        real dx, dy, dz;
        diff(a, b, rd, dx, dy, dz);
        return dx * dx + dy * dy + dz * dz < rd.rl2d;
    }
};

// The mixed form with 16-bit neighbour-list entries holding the neighbour's
// slot (its byte offset is the slot times 16): for contexts whose replicas
// all have at most 65536 atoms.  Half the list bytes of PMixed.
struct PMixed16 : PMixed {
    using entry_t = uint16_t;
    static constexpr bool kSlotEntries = true;
};

// The byte offset of a list entry's neighbour from the replica's first
// position.
template <class P>
__device__ __forceinline__ uint32_t entry_offset(uint32_t v)
{
    if constexpr (P::kSlotEntries)
        return v * (uint32_t)sizeof(typename P::pos_t);
    else
        return v;
}

// Entries are padded, per atom, with entries naming the atom itself up to a
// whole number of groups of 4 rows of tpa entries (at most the capacity M, a
// multiple of 32), so that the force loop reads whole groups without
// per-entry bounds; the self pair has r = 0 and is excluded by the force.
__host__ __device__ constexpr int padded_entries(int n, int tpa, int M)
{
    const int g = 4 * tpa;
    const int p = (n + g - 1) / g * g;
    return p < M ? p : M;
}

template <class P>
__device__ __forceinline__ void set_xyz(typename P::vel_t& v, typename P::real x, typename P::real y, typename P::real z)
{
    v.x = x;
    v.y = y;
    v.z = z;
}


// Rebuild requests.  An atom that has moved more than half the skin since
// the last list update requests an update before the force of step f by
// storing rebuild_tag(f) in the word of f's parity; the force of step f
// rebuilds when that word holds rebuild_tag(f).  A request is never cleared:
// the tags of other steps do not match, so no clear has to be ordered
// against the next step's requests.
__device__ __forceinline__ uint32_t rebuild_tag(int64_t f)
{
    return 0x80000000u | (uint32_t)(f & 0x7fffffff);
}

// ---------------------------------------------------------------------------
// Phase functions.  Each works on a range of atoms (or a whole replica) of
// replica r; the lockstep kernels and the persistent engine call them.

// First half of a step from a stopped boundary (B A O A of BAOAB; B A A
// without O under the velocity rescale) for atom slot i:
// v = alpha v + h F;  x += h v;  v = c1 v + c2 xi;  x += h v;
// then the half-skin test against x_ref, which sets the update flag of the
// next step's parity.  xi: Philox counter (atom id, step, replica, 1).
// (alpha: the velocity factor applied first, in FP64 as computed)
template <class P>
__device__ __forceinline__ void start_atom_scaled(const DevState& d, const StepArgs& sa, const RepDev& rd, int r,
                                                  int i, int cur, int64_t step, double alpha)
{
    using real = typename P::real;
    const int g = rd.base + i;
    typename P::pos_t* pos = P::pos(d, cur);
    typename P::pos_t x = pos[g];
    typename P::vel_t v = P::vel(d)[g];
    const typename P::vel_t f = P::frc(d)[g];
    const real hh = (real)sa.h;
    const real a = (real)alpha;
    const real c1 = (real)sa.c1;
    const real c2 = (real)d.c2[r];
    real vx = a * v.x + hh * f.x, vy = a * v.y + hh * f.y, vz = a * v.z + hh * f.z;
    x = P::drift(x, hh * vx, hh * vy, hh * vz, rd);
    if (sa.thermo == kThermoLangevin) {
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
    }
    x = P::drift(x, hh * vx, hh * vy, hh * vz, rd);
    pos[g] = x;
    set_xyz<P>(v, vx, vy, vz);
    P::vel(d)[g] = v;
    real dx, dy, dz;
    P::diff(x, P::xref(d)[g], rd, dx, dy, dz);
    if (dx * dx + dy * dy + dz * dz > P::lim2(rd))
        __hip_atomic_store(&d.flag[(size_t)((step + 1) & 1) * sa.R + r], rebuild_tag(step + 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <class P>
__device__ __forceinline__ void start_atom(const DevState& d, const StepArgs& sa, const RepDev& rd, int r, int i,
                                           int cur, int64_t step, bool apply_alpha)
{
    start_atom_scaled<P>(d, sa, rd, r, i, cur, step, apply_alpha ? d.alpha[r] : 1.0);
}

// Exclusive scan of the ncc cell counts in LDS with the whole workgroup, in
// place; cnt[ncc] := N.  Contiguous chunks per thread; the chunk sums are
// scanned within each wave by shuffles, then across the waves (`part`: 128
// ints of LDS).  Ends with a workgroup barrier.
__device__ __forceinline__ void cell_scan(int* cnt, int ncc, int N, int* part)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (ncc + nt - 1) / nt;
    const int c0 = tid * chunk, c1 = min(ncc, c0 + chunk);
    int s = 0;
    for (int c = c0; c < c1; ++c) s += cnt[c];
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    int x = s;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) part[wv] = x;
    __syncthreads();
    if (wv == 0) {
        int t = lane < nw ? part[lane] : 0;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(t, o, 64);
            if (lane >= o) t += y;
        }
        if (lane < nw) part[64 + lane] = t;
    }
    __syncthreads();
    int run = (wv > 0 ? part[64 + wv - 1] : 0) + x - s;
    for (int c = c0; c < c1; ++c) {
        const int n = cnt[c];
        cnt[c] = run;
        run += n;
    }
    if (tid == 0) cnt[ncc] = N;
    __syncthreads();
}

// Reorder with every atom held in registers (at most K per thread): one
// read of x and v, the arrival order in each cell from LDS atomics, the ids
// of each cell's atoms in LDS, and each atom's place in its cell the number
// of atoms of the cell with a smaller id; x, x_ref and v are then written in
// place at the new slots.
template <class P, int K>
__device__ void reorder_in_registers(const DevState& d, const RepDev& rd, int r, int cur, int* cnt, int* part)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nc = rd.ncell, ncc = nc * nc * nc, N = rd.N;
    typename P::pos_t* pos = P::pos(d, cur) + rd.base;
    typename P::vel_t* vel = P::vel(d) + rd.base;
    int* idk = cnt + ncc + 1;  // ids in (cell, arrival) order
    for (int c = tid; c < ncc; c += nt) cnt[c] = 0;
    __syncthreads();
    typename P::pos_t px[K];
    typename P::vel_t pv[K];
    int cc[K], ar[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int i = tid + j * nt;
        if (i < N) {
            px[j] = pos[i];
            pv[j] = vel[i];
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        cc[j] = 0;
        ar[j] = 0;
        if (tid + j * nt < N) {
            cc[j] = (P::cellc(px[j].x, rd) * nc + P::cellc(px[j].y, rd)) * nc + P::cellc(px[j].z, rd);
            ar[j] = atomicAdd(&cnt[cc[j]], 1);
        }
    }
    __syncthreads();
    cell_scan(cnt, ncc, N, part);
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (tid + j * nt < N) idk[cnt[cc[j]] + ar[j]] = P::id(px[j]);
    __syncthreads();
    int32_t* cstart = d.cell_start + rd.cell_base;
    for (int c = tid; c <= ncc; c += nt) cstart[c] = cnt[c];
    typename P::pos_t* xref = P::xref(d) + rd.base;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (tid + j * nt < N) {
            const int a = cnt[cc[j]], e = cnt[cc[j] + 1];
            const int myid = P::id(px[j]);
            int rk = 0;
            for (int m = a; m < e; ++m) rk += idk[m] < myid ? 1 : 0;
            pos[a + rk] = px[j];
            xref[a + rk] = px[j];
            vel[a + rk] = pv[j];
        }
    }
    if (tid == 0) d.rebuilds[r] += 1;
    __syncthreads();
}

// Reorder one replica by cell with the whole workgroup (blockDim a multiple
// of 64, at most 4096): counting sort of the atoms into the cell grid
// (counts in LDS), each cell then ordered by atom id so the result does not
// depend on scheduling; x_ref := x.  The other position buffer and the
// velocity scratch serve as gather space.  `cnt` holds kMaxCells + 1 ints of
// LDS; when the counts and three N-int scratch arrays fit there the scratch
// stays in LDS, otherwise it goes to the global per-atom arrays.
template <class P>
__device__ void reorder_replica(const DevState& d, const RepDev& rd, int r, int cur, int* cnt, int* part)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nc = rd.ncell, ncc = nc * nc * nc, N = rd.N;
    constexpr int K = P::kF64 ? 2 : 4;
    if (N <= K * nt && ncc + 1 + N <= kMaxCells + 1) {
        reorder_in_registers<P, K>(d, rd, r, cur, cnt, part);
        return;
    }
    typename P::pos_t* pos = P::pos(d, cur) + rd.base;
    typename P::pos_t* tmp = P::pos(d, cur ^ 1) + rd.base;
    typename P::vel_t* vel = P::vel(d) + rd.base;
    typename P::vel_t* velt = P::velt(d) + rd.base;
    const bool in_lds = ncc + 1 + 3 * N <= kMaxCells + 1;
    int32_t* cellid = in_lds ? cnt + ncc + 1 : d.cellid + rd.base;
    int32_t* rank = in_lds ? cellid + N : d.rank + rd.base;
    int32_t* perm = in_lds ? rank + N : d.perm + rd.base;
    for (int c = tid; c < ncc; c += nt) cnt[c] = 0;
    __syncthreads();
    for (int i = tid; i < N; i += nt) {
        const typename P::pos_t p = pos[i];
        const int c = (P::cellc(p.x, rd) * nc + P::cellc(p.y, rd)) * nc + P::cellc(p.z, rd);
        cellid[i] = c;
        rank[i] = atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    cell_scan(cnt, ncc, N, part);
    int32_t* cstart = d.cell_start + rd.cell_base;
    for (int c = tid; c <= ncc; c += nt) cstart[c] = cnt[c];
    for (int i = tid; i < rd.N; i += nt) perm[cnt[cellid[i]] + rank[i]] = i;
    __syncthreads();
    // order every cell by atom id: the ids in cell order go to the free
    // `cellid` scratch; each atom's place in its cell is the number of atoms
    // of the cell with a smaller id.  The ordered slots go to `rank`.
    for (int k = tid; k < N; k += nt) cellid[k] = P::id(pos[perm[k]]);
    __syncthreads();
    for (int k = tid; k < N; k += nt) {
        int lo = 0, hi = ncc - 1;  // the cell of sorted slot k
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cnt[mid] <= k)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int a = cnt[lo], e = cnt[lo + 1];
        const int myid = cellid[k];
        int rk = 0;
        for (int m = a; m < e; ++m) rk += cellid[m] < myid ? 1 : 0;
        rank[a + rk] = perm[k];
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
    __syncthreads();
}

// Rows of the list build scanned by lane q of an LPA-lane group (nc >= 5):
// the 25 rows (x offset major) dealt out so that every lane expects about
// the same number of candidate cells after trimming (centre rows reach
// about 4.6 cells, edge rows 2.6, corner rows 0.5).  -1: no row.  Packed as
// 5 bits per lane per slot w.
template <int LPA>
struct ListRowSets;
template <>
struct ListRowSets<8> {
    static constexpr int kRPL = 4;
    static constexpr int8_t rows[8][4] = {{3, 12, 21, -1}, {0, 7, 10, 20}, {4, 11, 14, 24}, {5, 9, 13, -1},
                                          {15, 17, 19, -1}, {6, 18, -1, -1}, {2, 8, 23, -1}, {1, 16, 22, -1}};
};
template <>
struct ListRowSets<4> {
    static constexpr int kRPL = 7;
    static constexpr int8_t rows[4][7] = {{1, 5, 9, 12, 16, 22, -1}, {0, 7, 10, 15, 17, 19, 20},
                                          {3, 6, 11, 18, 23, -1, -1}, {2, 4, 8, 13, 14, 21, 24}};
};
template <int LPA>
__host__ __device__ constexpr uint64_t list_row_pack(int w)
{
    uint64_t v = 0;
    for (int q = 0; q < LPA; ++q) v |= (uint64_t)(ListRowSets<LPA>::rows[q][w] & 31) << (5 * q);
    return v;
}
// LDS words per lane that list_rows needs (range starts, slot offsets, end)
template <int LPA>
__host__ __device__ constexpr int list_lds_words()
{
    return 4 * ListRowSets<LPA>::kRPL + 1;
}

// Verlet list build on the fine cell grid (cell side >= half the list
// radius, cells ordered z fastest): the candidates of an atom are the atoms
// of the 5 x 5 x 5 cells around its own, i.e. 25 rows of 5 consecutive
// cells, each row one or two contiguous slot ranges of the cell-sorted
// arrays (all nc^2 columns of nc cells when there are fewer than 5 cells
// per side).  Every row is first trimmed to the atom's own position: it is
// skipped when its column lies farther than the list radius in x-y, and
// otherwise shortened to the z cells that reach within the radius
// (conservative bounds with a 1e-4 margin: no pair within the list radius is
// lost).  A group of LPA lanes serves one atom; lane q takes a fixed set of
// rows and scans their candidates as one flat sequence, four in flight (the
// slot of flat candidate k is k plus the offset of its range, found from a
// bit mask of range starts and a small per-lane table in LDS).  Hits are
// kept as a bit mask; a scan of the lane counts over the group places them,
// so the list holds lane 0's hits, then lane 1's, ..., each in scan order.
// Entry k of atom i lives at nl[nl_base + ((k / tpa) Np + i) tpa + k % tpa]
// (tpa a power of two) and holds the byte offset of the neighbour's position
// from the replica's first slot.  The distance test is P::list_close on list
// keys.  `pos`: the replica's positions (global); `keys`: the candidates'
// keys (P::key_t, e.g. a copy in LDS) or their positions (P::pos_t, keys made
// on the fly); `cs`: the replica's cell starts (global or a copy in LDS).
// `lds`: list_lds_words<LPA>() words of this lane.
template <class P, int LPA, class Src>
__device__ __forceinline__ void list_rows(const DevState& d, const RepDev& rd, const typename P::pos_t* pos,
                                          const Src* keys, const int32_t* cs, int i, bool act, int q, int tpa, int M,
                                          int* lds)
{
    constexpr int RPL = ListRowSets<LPA>::kRPL;
    const int nc = rd.ncell;
    const typename P::pos_t pi = pos[act ? i : 0];
    const typename P::key_t ki = P::list_key(pi);
    // this lane's ranges: flat start lds[2 n], slot offset lds[2 n + 1]
    int T = 0, nr = 0;
    uint64_t bounds = 0;  // bit k: a range other than the first starts at flat index k
    lds[1] = 0;           // offset used by a lane without candidates
    // (an empty range writes slot nr, which the next range or the end mark
    // overwrites: at most 2 RPL ranges, so every write stays in the lane's
    // 4 RPL + 1 words)
    auto add = [&](int a, int b) {
        const bool ne = b > a;
        if (ne && nr > 0 && T < 64) bounds |= 1ull << T;
        lds[2 * nr] = T;
        lds[2 * nr + 1] = a - T;
        nr += ne ? 1 : 0;
        T += ne ? b - a : 0;
    };
    if (act) {
        const int cx = P::cellc(pi.x, rd), cy = P::cellc(pi.y, rd), cz = P::cellc(pi.z, rd);
        // offsets inside the own cell, in cell units
        const float fx = fminf(fmaxf(P::cellpos(pi.x, rd) - (float)cx, 0.f), 1.f);
        const float fy = fminf(fmaxf(P::cellpos(pi.y, rd) - (float)cy, 0.f), 1.f);
        const float fz = fminf(fmaxf(P::cellpos(pi.z, rd) - (float)cz, 0.f), 1.f);
        if (nc >= 5) {
            // every row slot gives two ranges of cell starts, [cs[ca], cs[cb])
            // then [cs[cc], cs[cd]) (empty when unused), so that all loads of
            // cell starts are issued before the first range is written
            int ca[RPL], cb[RPL], cc[RPL], cd[RPL];
#pragma unroll
            for (int w = 0; w < RPL; ++w) {
                const int row = (int)((list_row_pack<LPA>(w) >> (5 * q)) & 31u);  // 31: no row
                const int ox = row / 5 - 2, oy = row % 5 - 2;
                // distance from the atom to the row's column, in cell units
                const float ex = ox > 0 ? (float)ox - fx : (ox < 0 ? fx + (float)(-ox - 1) : 0.f);
                const float ey = oy > 0 ? (float)oy - fy : (oy < 0 ? fy + (float)(-oy - 1) : 0.f);
                const float h2 = rd.rlcell2 - ex * ex - ey * ey;
                const bool use = row < 25 && h2 > 0.f;
                int x = cx + ox, y = cy + oy;
                x += x < 0 ? nc : 0;
                x -= x >= nc ? nc : 0;
                y += y < 0 ? nc : 0;
                y -= y >= nc ? nc : 0;
                const int rb = (x * nc + y) * nc;
                const float h = sqrtf(fmaxf(h2, 0.f));
                const int z0 = cz + max(-2, (int)floorf(fz - h)), z1 = cz + min(2, (int)floorf(fz + h));
                // z cells z0..z1, wrapped: below 0 the top cells come first,
                // past nc - 1 the bottom cells come second
                const bool lo = z0 < 0, hi = z1 >= nc;
                ca[w] = rb + (lo ? z0 + nc : z0);
                cb[w] = use ? rb + (lo || hi ? nc : z1 + 1) : ca[w];
                cc[w] = rb;
                cd[w] = rb + (use ? (lo ? z1 + 1 : (hi ? z1 - nc + 1 : 0)) : 0);
            }
            int va[RPL], vb[RPL], vc[RPL], vd[RPL];
#pragma unroll
            for (int w = 0; w < RPL; ++w) {
                va[w] = cs[ca[w]];
                vb[w] = cs[cb[w]];
                vc[w] = cs[cc[w]];
                vd[w] = cs[cd[w]];
            }
#pragma unroll
            for (int w = 0; w < RPL; ++w) {
                add(va[w], vb[w]);
                add(vc[w], vd[w]);
            }
        } else {
#pragma unroll
            for (int w = 0; w < RPL; ++w) {
                const int row = q + w * LPA;
                if (row < nc * nc) add(cs[row * nc], cs[row * nc + nc]);
            }
        }
    }
    lds[2 * nr] = T;
    auto test = [&](const Src& kj, int j) {
        // bitwise, so that no load is moved under a branch
        return P::list_close(ki, P::list_key(kj), rd) & (j != i);
    };
    // keys by 32-bit byte offsets from the replica's base
    const char* kbase = reinterpret_cast<const char*>(keys);
    auto load = [&](uint32_t j) { return *reinterpret_cast<const Src*>(kbase + j * (uint32_t)sizeof(Src)); };
    const int T64 = T < 64 ? T : 64;
    uint64_t mk = 0;
    int cnt = 0;
    int ri = 0;  // ranges started at flat indices 1..k0
    for (int k0 = 0; k0 < T64; k0 += 4) {
        // the range of candidates k0 .. k0 + 3 from the range-start bits
        // above k0; the slot of flat candidate k is k plus its range's offset
        // (a candidate past the lane's end reads at most three slots past the
        // last range, inside the position arrays' slack, and is masked out)
        const uint32_t w = (uint32_t)(bounds >> (k0 + 1));
        int rr[4];
        rr[0] = ri;
        rr[1] = rr[0] + (int)(w & 1u);
        rr[2] = rr[1] + (int)((w >> 1) & 1u);
        rr[3] = rr[2] + (int)((w >> 2) & 1u);
        ri = rr[3] + (int)((w >> 3) & 1u);
        uint32_t jj[4];
        Src pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) jj[u] = (uint32_t)(k0 + u + lds[2 * rr[u] + 1]);
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = load(jj[u]);
        uint32_t nib = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) nib |= test(pj[u], (int)jj[u]) ? (1u << u) : 0u;
        mk |= (uint64_t)nib << k0;
    }
    // candidates past the lane's end (the last group of four) are dropped
    if (T64 < 64) mk &= (1ull << T64) - 1ull;
    cnt = __popcll(mk);
    // candidates past the mask (only with very full rows): walk the ranges
    auto walk = [&](auto&& on_hit) {
        for (int n = 0; n < nr; ++n) {
            const int k1 = lds[2 * n + 2], off = lds[2 * n + 1];
            for (int k = max(lds[2 * n], 64); k < k1; ++k)
                if (test(load((uint32_t)(k + off)), k + off)) on_hit(k + off);
        }
    };
    if (T > 64) walk([&](int) { ++cnt; });
    // first entry of this lane: the hits of the lanes before it (an
    // inclusive scan over the group by row shifts; the groups of LPA lanes
    // are aligned within the 16-lane rows, and a lane takes no value from
    // below its group's first lane)
    // (each shift runs in every lane of the wave, outside any condition: a
    // lane switched off would hand `old` to the lane above it)
    static_assert(LPA == 4 || LPA == 8, "list-build groups of 4 or 8 lanes");
    int incl = cnt;
    const int s1 = __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, false);  // row_shr:1
    incl += q >= 1 ? s1 : 0;
    const int s2 = __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, false);  // row_shr:2
    incl += q >= 2 ? s2 : 0;
    if constexpr (LPA == 8) {
        const int s4 = __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, false);  // row_shr:4
        incl += q >= 4 ? s4 : 0;
    }
    int o = incl - cnt;
    // entry o of atom i: element ((o / tpa) Np + i) tpa + o % tpa of the
    // list (tpa a power of two)
    using E = typename P::entry_t;
    E* nl = reinterpret_cast<E*>(d.nl) + rd.nl_base;
    const int ltpa = __builtin_ctz((unsigned)tpa);
    const uint32_t jump = (uint32_t)rd.Np * (uint32_t)tpa - (uint32_t)(tpa - 1);
    uint32_t e = ((uint32_t)o >> ltpa) * (uint32_t)rd.Np * (uint32_t)tpa + (uint32_t)i * (uint32_t)tpa +
                 (uint32_t)(o & (tpa - 1));
    // the entry of slot j: the slot itself, or its byte offset
    auto value = [&](int j) -> E {
        if constexpr (P::kSlotEntries)
            return (E)j;
        else
            return (E)((uint32_t)j * (uint32_t)sizeof(typename P::pos_t));
    };
    auto put = [&](int j) {
        if ((unsigned)o < (unsigned)M) nl[e] = value(j);
        ++o;
        e += (o & (tpa - 1)) ? 1u : jump;
    };
    // hits in flat order; the range of hit k from the range starts at 1..k
    uint32_t mlo = (uint32_t)mk, mhi = (uint32_t)(mk >> 32);
    const uint32_t blo = (uint32_t)bounds, bhi = (uint32_t)(bounds >> 32);
    while (mlo) {
        const int k = __builtin_ctz(mlo);
        mlo &= mlo - 1u;
        put(k + lds[2 * __popc(blo & ((2u << k) - 1u)) + 1]);
    }
    const int rhi = __popc(blo);
    while (mhi) {
        const int k = __builtin_ctz(mhi);
        mhi &= mhi - 1u;
        put(32 + k + lds[2 * (rhi + __popc(bhi & ((2u << k) - 1u))) + 1]);
    }
    if (T > 64) walk(put);
    // the group's last lane holds the total; it pads the atom's entries
    // with self entries to whole groups of rows
    if (act && q == LPA - 1) {
        const int n = incl < M ? incl : M;
        d.nn[rd.base + i] = n;
        if (incl > M) atomicOr(d.overflow, 1u);
        const int np = padded_entries(n, tpa, M);
        for (int k = n; k < np; ++k)
            nl[((uint32_t)k >> ltpa) * (uint32_t)rd.Np * (uint32_t)tpa + (uint32_t)i * (uint32_t)tpa +
               (uint32_t)(k & (tpa - 1))] = value(i);
    }
}

// LJ force (+ energy) on atom slot ia over its Verlet list, TPA lanes per
// atom (lane q takes entries q, q + TPA, ...), summed over the TPA lanes:
// every lane of the group ends with the sums (grid units in the mixed form)
// and the atom's position pi.  `pos`: the replica's positions (global or an
// LDS copy).
// u(r) = 4 (r^-12 - r^-6) - u(r_c), F_i = 24 (2 r^-14 - r^-8) r_ij for r < r_c
// (Example section: cutoff 2.5; energy shifted, force truncated).  Every
// lane of the TPA group must call this (the reduction shuffles).
template <class P, int MODE, int TPA>
__device__ __forceinline__ void force_sum(const DevState& d, const StepArgs& sa, const RepDev& rd,
                                          const typename P::pos_t* pos, int ia, int q, bool valid,
                                          typename P::pos_t& pi, typename P::real& fx, typename P::real& fy,
                                          typename P::real& fz, typename P::real& e)
{
    using real = typename P::real;
    constexpr bool kEnergy = (MODE == kStopEnergy || MODE == kQuery || MODE == kRefresh);
    fx = 0;
    fy = 0;
    fz = 0;
    e = 0;
    pi = typename P::pos_t{};
    if (valid) {
        const char* pb = reinterpret_cast<const char*>(pos);
        pi = pos[ia];
        const int nnb = d.nn[rd.base + ia];
        // list row kk of this lane: the replica's row base (the same for the
        // whole wave) plus the lane's 32-bit byte offset; rows past the
        // atom's entries up to a whole group of 4 hold the atom itself
        using E = typename P::entry_t;
        const char* __restrict__ nlb = reinterpret_cast<const char*>(reinterpret_cast<const E*>(d.nl) + rd.nl_base);
        const uint32_t eo = (uint32_t)(ia * TPA + q) * (uint32_t)sizeof(E);
        const size_t rowb = (size_t)rd.Np * TPA * sizeof(E);
        const int nrow = padded_entries(nnb, TPA, sa.M) / TPA;
        if constexpr (P::kF64) {
            auto entry = [&](int kk) { return (uint32_t)*reinterpret_cast<const E*>(nlb + (size_t)kk * rowb + eo); };
            const double rc2 = rd.rc2d;
            for (int kk = 0; kk < nrow; ++kk) {
                const typename P::pos_t pj = *reinterpret_cast<const typename P::pos_t*>(pb + entry(kk));
                double dx, dy, dz;
                P::diff(pi, pj, rd, dx, dy, dz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2 && r2 > 0.0) {  // (r = 0: the atom itself)
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
            // one pair; the atom itself (r = 0, a padding entry) is excluded
            auto pair = [&](const int4& pj) {
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
                in = in && r2 > 0.0f;
                const float ir2 = __builtin_amdgcn_rcpf(r2) * is2;
                const float ir6 = ir2 * ir2 * ir2;
                const float ff = in ? ir2 * ir6 * __builtin_fmaf(48.0f, ir6, -24.0f) : 0.0f;
                fx = __builtin_fmaf(ff, dx, fx);
                fy = __builtin_fmaf(ff, dy, fy);
                fz = __builtin_fmaf(ff, dz, fz);
                if constexpr (kEnergy) e += in ? __builtin_fmaf(4.0f * ir6, ir6, -4.0f * ir6) - ushift : 0.0f;
            };
            // four neighbours in flight: the entries of the next four rows are
            // loaded while the current four pairs are computed (the loads of
            // the group after the last are past the atom's rows; their values
            // are not used)
            constexpr int U = 4;
            // the list words through a buffer resource over the replica's
            // block: the row offset goes in a scalar register and the lane's
            // in a 32-bit vector register, so an entry load needs no vector
            // address arithmetic (the host keeps a block under 2^32 bytes;
            // loads past the block return 0)
            const __amdgpu_buffer_rsrc_t nlr = __builtin_amdgcn_make_buffer_rsrc(
                (void*)nlb, (short)0, (int)((uint32_t)rd.Np * (uint32_t)sa.M * (uint32_t)sizeof(E)),
                0x00020000);  // (descriptor word 3 of gfx9: 32-bit elements)
            const uint32_t rowb32 = (uint32_t)rowb;
            auto bentry = [&](int kk) -> uint32_t {
                if constexpr (sizeof(E) == 2)
                    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(nlr, (int)eo, (int)((uint32_t)kk * rowb32), 0);
                else
                    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(nlr, (int)eo, (int)((uint32_t)kk * rowb32), 0);
            };
            uint32_t jn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) jn[u] = entry_offset<P>(bentry(u));
            for (int kk = 0; kk < nrow; kk += U) {
                int4 pj[U];
#pragma unroll
                for (int u = 0; u < U; ++u) pj[u] = *reinterpret_cast<const int4*>(pb + jn[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) jn[u] = entry_offset<P>(bentry(kk + U + u));
#pragma unroll
                for (int u = 0; u < U; ++u) pair(pj[u]);
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
}

// The step epilogue of atom slot ia from its force sums (force_sum), by
// MODE:
//   kFused:      v += h F (ends this step), v += h F, x += h v, O, x += h v
//                (the next step's first half; positions to the other buffer)
//   kStop/kStopEnergy: v += h F; store F (and the per-atom energy)
//   kQuery:      F and energy to the query buffer in atom-id order only
//   kRefresh:    store F and the per-atom energy; velocities untouched.
// (v0: the atom's velocity, xr0: its x_ref (read in kFused only), both
// loaded by the caller)
template <class P, int MODE>
__device__ __forceinline__ void force_epilogue_v(const DevState& d, const StepArgs& sa, const RepDev& rd, int r,
                                                 int ia, int cur, int64_t step_next, int par,
                                                 const typename P::pos_t& pi, typename P::real fx,
                                                 typename P::real fy, typename P::real fz, typename P::real e,
                                                 typename P::vel_t v0, const typename P::pos_t& xr0)
{
    using real = typename P::real;
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
    } else {
        const real hh = MODE == kRefresh ? (real)0 : (real)sa.h;
        typename P::vel_t v = v0;
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
            P::diff(x, xr0, rd, dx, dy, dz);
            if (dx * dx + dy * dy + dz * dz > P::lim2(rd))
                __hip_atomic_store(&d.flag[(size_t)(par ^ 1) * sa.R + r], rebuild_tag(step_next + 1),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
            if constexpr (MODE == kStop || MODE == kStopEnergy) {
                // the atom's terms of the velocity rescale at this boundary:
                // v.v and its squared normals of the chi-square sum (Philox
                // counter (atom id, step, replica, purpose 4); all three but
                // for atom 0, whose first normal is R1, and atom 1, whose
                // first is left out: 3N - 4 terms in all)
                if (sa.thermo == kThermoSVR) {
                    const int id = P::id(pi);
                    double z0, z1, z2;
                    normals3d(draw(sa.seed, (uint32_t)id, (uint32_t)step_next, (uint32_t)r, kPurposeSVR), z0, z1, z2);
                    const double chi =
                        (id == 0 ? 0.0 : (id == 1 ? 0.0 : z0 * z0)) + (id == 0 ? 0.0 : z1 * z1 + z2 * z2);
                    d.svrq[g] = make_double2((double)vx * (double)vx + (double)vy * (double)vy + (double)vz * (double)vz,
                                             chi);
                }
            }
        }
    }
}

// The epilogue with the atom's velocity and x_ref loaded here.
template <class P, int MODE>
__device__ __forceinline__ void force_epilogue(const DevState& d, const StepArgs& sa, const RepDev& rd, int r, int ia,
                                               int cur, int64_t step_next, int par, const typename P::pos_t& pi,
                                               typename P::real fx, typename P::real fy, typename P::real fz,
                                               typename P::real e)
{
    typename P::vel_t v{};
    typename P::pos_t xr{};
    if constexpr (MODE != kQuery) v = P::vel(d)[rd.base + ia];
    if constexpr (MODE == kFused) xr = P::xref(d)[rd.base + ia];
    force_epilogue_v<P, MODE>(d, sa, rd, r, ia, cur, step_next, par, pi, fx, fy, fz, e, v, xr);
}

// Force sum and epilogue of atom slot ia by the TPA lanes of its group (the
// epilogue on lane 0).
template <class P, int MODE, int TPA>
__device__ __forceinline__ void force_atom(const DevState& d, const StepArgs& sa, const RepDev& rd, int r, int ia,
                                           int q, bool valid, int cur, int64_t step_next, int par)
{
    typename P::pos_t pi;
    typename P::real fx, fy, fz, e;
    force_sum<P, MODE, TPA>(d, sa, rd, P::pos(d, cur) + rd.base, ia, q, valid, pi, fx, fy, fz, e);
    if (!valid || q != 0) return;
    force_epilogue<P, MODE>(d, sa, rd, r, ia, cur, step_next, par, pi, fx, fy, fz, e);
}

// Replica reductions sum over kRedWidth fixed slices (atom slots i = q mod
// kRedWidth, in slot order) and then a fixed pairwise tree, so the result
// does not depend on the workgroup size (the lockstep and the persistent
// engine give the same bits).
constexpr int kRedWidth = 256;
// LDS doubles a replica reduction needs: two arrays of kRedWidth partial
// sums and two values of the velocity rescale
constexpr int kRedLds = 2 * kRedWidth + 2;

// Slice sums of f(i) (one or two components) over the atom slots of replica
// rd: slice q = sum over i = q, q + kRedWidth, ... < N in slot order, with
// every thread's loads issued eight at a time, each round before its
// additions (sixteen in flight cost the persistent kernel's step loop
// register spills).  Slice q goes to a[q] (and b[q]).  Workgroup barrier at
// the end.
template <int C, class F>
__device__ __forceinline__ void slice_sums(int N, F f, double* a, double* b)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int q = tid; q < kRedWidth; q += nt) {
        double s0 = 0.0, s1 = 0.0;
        int i = q;
        for (; i < N; i += 8 * kRedWidth) {
            double2 t[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) t[k] = i + k * kRedWidth < N ? f(i + k * kRedWidth) : make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (i + k * kRedWidth < N) {  // (the same additions in the same order)
                    s0 += t[k].x;
                    if constexpr (C == 2) s1 += t[k].y;
                }
            }
        }
        a[q] = s0;
        if constexpr (C == 2) b[q] = s1;
    }
    __syncthreads();
}

// The fixed pairwise tree over kRedWidth slice sums: a[q] += a[q + off] for
// off = kRedWidth/2, ..., 1, all in the first wave (its lane l holds slices
// l, l + 64, l + 128, l + 192, which makes the first two levels additions in
// registers; the last six are shuffles), pairing the same elements in the
// same order.  The total is returned to thread 0 (other threads:
// unspecified).  Needs a workgroup of at least 64 threads and the slice
// sums' workgroup barrier before it.
template <int C>
__device__ __forceinline__ void tree_sums(const double* a, const double* b, double& ta, double& tb)
{
    static_assert(kRedWidth == 256, "the tree assumes four slices per lane");
    const int tid = threadIdx.x;
    ta = 0.0;
    tb = 0.0;
    if (tid < 64) {
        double va = (a[tid] + a[tid + 128]) + (a[tid + 64] + a[tid + 192]), vb = 0.0;
        if constexpr (C == 2) vb = (b[tid] + b[tid + 128]) + (b[tid + 64] + b[tid + 192]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ua = __shfl_down(va, off, 64);
            va = tid < off ? va + ua : va;
            if constexpr (C == 2) {
                const double ub = __shfl_down(vb, off, 64);
                vb = tid < off ? vb + ub : vb;
            }
        }
        ta = va;
        tb = vb;
    }
}

// R1 of the velocity rescale of replica r at step boundary s: the first
// normal of atom 0's draw (Philox counter (0, s, r, purpose 4)).
__device__ __forceinline__ double svr_normal(uint64_t seed, int64_t s, int r)
{
    double z0, z1, z2;
    normals3d(draw(seed, 0u, (uint32_t)s, (uint32_t)r, kPurposeSVR), z0, z1, z2);
    return z0;
}

// Stochastic velocity rescale of replica r at step boundary s (Example
// section: the thermostat; Bussi, Donadio and Parrinello 2007), computed by
// one workgroup (part: kRedLds doubles) after a stopping force phase has
// left each atom's terms in svrq: K = sum v.v / 2 and the chi-square sum S of
// N_f - 1 = 3N - 4 squared normals, both in FP64 (fixed slice order); R1 is
// the first normal of atom 0 (Philox counter (0, s, r, purpose 4)); then
//   K' = K + (1 - c)(Kbar (R1^2 + S) / N_f - K) + 2 R1 sqrt(c (1 - c) K Kbar / N_f),
// Kbar = N_f T / 2 at the replica's temperature.  Returns the velocity
// factor sqrt(K'/K) (1 when K = 0) to every thread; the fixed order gives
// every workgroup that computes it the same bits.  R1 is given to thread 0
// (r1_known) or drawn here; the last thread draws it and reads the
// temperature the replica holds while the others load.  Ends with a
// workgroup barrier.
template <class P>
__device__ double svr_factor(const DevState& d, const RepDev& rd, int r, int64_t s, uint64_t seed, double c,
                             bool r1_known, double R1, double* part)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const double Nf = 3.0 * rd.N - 3.0;
    if (tid == nt - 1) {
        if (!r1_known) part[2 * kRedWidth] = svr_normal(seed, s, r);
        part[2 * kRedWidth + 1] = d.Tl[d.slot[r]];
    }
    const double2* q2 = d.svrq + rd.base;
    slice_sums<2>(rd.N, [&](int i) { return q2[i]; }, part, part + kRedWidth);
    double k2, chi;
    tree_sums<2>(part, part + kRedWidth, k2, chi);
    if (tid == 0) {
        const double K = 0.5 * k2, S = chi;
        if (!r1_known) R1 = part[2 * kRedWidth];
        const double Kbar = 0.5 * Nf * part[2 * kRedWidth + 1];
        double f = 1.0;
        if (K > 0.0) {
            const double Kn = K + (1.0 - c) * (Kbar * (R1 * R1 + S) / Nf - K) + 2.0 * R1 * sqrt(c * (1.0 - c) * K * Kbar / Nf);
            f = sqrt(Kn / K);
        }
        part[1] = f;
    }
    __syncthreads();
    const double f = part[1];
    __syncthreads();
    return f;
}

// The velocity rescale of svr_factor folded into the replica's pending
// velocity factor (alpha *= sqrt(K'/K)), by one workgroup.
template <class P>
__device__ void svr_replica(const DevState& d, const RepDev& rd, int r, int64_t s, uint64_t seed, double c,
                            bool r1_known, double R1, double* part)
{
    const double a = d.alpha[r];  // (loaded before the reduction's barriers)
    const double f = svr_factor<P>(d, rd, r, s, seed, c, r1_known, R1, part);
    if (threadIdx.x == 0) d.alpha[r] = a * f;
    __syncthreads();
}

// Potential energy of replica r in FP64 with the whole workgroup (part:
// kRedLds doubles): U = (1/2) sum_i e_i over the per-atom energies, in the
// fixed slice and tree order, stored to d.U[r] and returned to thread 0
// (other threads: unspecified).
template <class P>
__device__ double energy_replica(const DevState& d, const RepDev& rd, int r, double* part)
{
    const typename P::real* e = P::epot(d) + rd.base;
    slice_sums<1>(rd.N, [&](int i) { return make_double2((double)e[i], 0.0); }, part, nullptr);
    double u, unused;
    tree_sums<1>(part, nullptr, u, unused);
    if (threadIdx.x == 0) d.U[r] = 0.5 * u;
    __syncthreads();
    return 0.5 * u;
}

}  // namespace re
