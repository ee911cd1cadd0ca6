// re_internal.hpp -- structures shared by the host runtime (re_host.cpp) and
// the device code (re_kernels.hip) of the replica-exchange LJ engine.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace re {

constexpr int kMaxCellsPerSide = 32;               // cell grid cap (cells may exceed r_list/2)
constexpr int kMaxCells = kMaxCellsPerSide * kMaxCellsPerSide * kMaxCellsPerSide;
constexpr int kReorderThreads = 1024;              // one workgroup per replica
constexpr int kPersistLdsWords = 36864;            // persistent kernel's shared int array (144 KiB)
#ifndef RE_LIST_LANES
#define RE_LIST_LANES 8
#endif
constexpr int kListLanes = RE_LIST_LANES;          // list-build lanes per atom (4 or 8)
constexpr int kPosSlack = 64;                      // position slots past the last replica (list-build reads)
constexpr int kListSlackRows = 8;                  // list rows read past a replica's block by the
                                                   // force loop's prefetch (values unused)
constexpr uint32_t kPurposeInitVel = 0u;           // Philox counter word 3 ("purpose")
constexpr uint32_t kPurposeOStep = 1u;
constexpr uint32_t kPurposeExchange = 2u;
constexpr uint32_t kPurposeVacancy = 3u;
constexpr uint32_t kPurposeSVR = 4u;
constexpr uint32_t kPurposePattern = 5u;
constexpr int kThermoLangevin = 0;                 // BAOAB Langevin
constexpr int kThermoSVR = 1;                      // velocity Verlet + stochastic velocity rescale

// Per-replica constants, in device memory (one record per replica).
// "pair units": the mixed form measures pair vectors in grid units of the
// 32-bit fixed-point box (s = L 2^-32 per unit); the FP64 form in LJ units
// (s = 1).
struct RepDev {
    int32_t N;          // atoms
    int32_t base;       // first atom slot in the concatenated arrays (multiple of 64)
    int32_t ncell;      // cells per side
    int32_t cell_base;  // first entry of this replica in the cell arrays (ncell^3 + 1 entries)
    int64_t nl_base;    // first element of this replica's neighbour list
    int32_t Np;         // N rounded up to a multiple of 64 (list row length)
    int32_t tpa;        // lanes per atom of this replica's force pass and list layout (1, 2, 4, 8)
    float rlcell2;      // (list radius / cell side)^2 with a 1e-4 margin: row trimming
    double L;           // box side
    double s;           // length of one pair unit (mixed: L 2^-32; FP64: 1)
    double inv_s;       // 1 / s
    float sf, inv_sf;   // the same in FP32
    float inv_s2f;      // 1 / s^2 in FP32
    float rc2f;         // r_c^2 in pair units (FP32)
    float near_lo, near_hi; // FP32 band around rc2f where the exact test decides
    float lim2f;        // (skin/2)^2 in pair units (FP32)
    uint32_t rl2q;      // mixed list build: (list radius in units of L 2^-16 + sqrt 3)^2, rounded up
    uint64_t rc2_exact; // ceil((r_c/s)^2): exact integer cutoff test (mixed)
    double rc2d, rl2d, lim2d; // FP64 versions (FP64 form, pair units = LJ units)
};

// One exchange record, laid out as re_xlog_rec of the C ABI.
struct XRec {
    int64_t attempt;
    int32_t master, slot_lo, rep_a, rep_b;
    int64_t step_a, step_b;
    double U_a, U_b, T_a, T_b, u;
    int32_t accepted, slot_hi;
};

// Device arrays of one context (all replicas concatenated).
struct DevState {
    // per atom; the mixed form uses the i/f arrays, the FP64 form the d arrays
    int4* posi[2];      // fixed-point positions, .w = atom id (ping-pong)
    float4* velf;       // velocities
    float4* frcf;       // forces at the last stopped step boundary
    int4* xrefi;        // positions at the last list update
    float* epotf;       // per-atom energy (sum over the atom's pairs)
    float4* veltf;      // reorder scratch
    double4* posd[2];   // FP64 positions, .w = atom id
    double4* veld;
    double4* frcd;
    double4* xrefd;
    double* epotd;
    double2* svrq;      // velocity rescale: per atom v.v and its chi-square terms at the last stop
    int32_t* wtab;      // work table of the replicas whose lists are rebuilt (lockstep), 4 R + 4 ints
    double4* veltd;
    // neighbour machinery
    int32_t* perm;      // reorder scratch: new slot -> old slot
    int32_t* cellid;    // reorder scratch
    int32_t* rank;      // reorder scratch
    int32_t* cell_start;// per replica ncell^3 + 1
    void* nl;           // neighbour lists (entries of the precision policy's entry_t)
    int32_t* nn;        // neighbours per atom
    // per replica
    RepDev* rep;
    int32_t* slot;      // ladder slot held by each replica
    double* Tl;         // ladder temperatures
    double* c2;         // Langevin noise amplitude for the temperature held
    double* alpha;      // velocity factor of the last exchange
    double* U;          // potential energy at the last stopped boundary
    uint32_t* flag;     // 2 x R list-update requests (by step parity; rebuild_tag of the step)
    int64_t* rebuilds;
    int64_t* steps;
    int64_t* attempts;  // per ladder pair
    int64_t* accepts;
    XRec* log;          // ring of exchange records
    int64_t* log_count; // records written so far
    uint32_t* overflow; // nonzero: a list or cell exceeded its capacity
    // scratch for queries
    double* fq;         // 4 doubles per atom
};

// Block tables of the wide kernels: block b works on replica rep[b] (or
// nothing when rep[b] < 0), atoms a0[b] .. a0[b] + atoms_per_block - 1.
struct BlockTable {
    int32_t* rep;
    int32_t* a0;
};

struct LaunchCfg {
    int block;      // threads per block of the wide kernels
    int tpa;        // force-kernel lanes per atom; 0: per replica (RepDev::tpa)
    int M;          // neighbour-list capacity per atom (a multiple of 32)
    int n16;        // mixed form: 16-bit list entries
    int64_t log_cap;
};

// Arguments of one launch of the step kernels.
struct StepArgs {
    int cur;          // position buffer holding the current positions
    int par;          // parity of the list-update requests read by this launch
    int R;            // replicas in the context
    int r0;           // first replica (per-replica kernels)
    int blk_off;      // first block-table entry (wide kernels)
    int block;        // threads per block (wide kernels)
    int tpa;          // force-kernel lanes per atom; 0: per replica (RepDev::tpa)
    int M;            // neighbour-list capacity per atom (a multiple of 32)
    int n16;          // mixed form: 16-bit list entries (every replica <= 65536 atoms)
    int force_all;    // reorder/list: ignore the flags
    int apply_alpha;  // start: multiply v by the last exchange factor
    BlockTable tab;   // block table of the wide kernels
    int64_t step;     // start: steps done; force (fused): steps done after this force
    double h;         // dt / 2
    double c1;        // exp(-gamma dt)
    double ushiftd;   // u_LJ(r_c)
    uint64_t seed;    // Philox key
    int thermo;       // kThermoLangevin | kThermoSVR
    int do_u;         // replica reduction: potential energy
    int do_svr;       // replica reduction: velocity rescale factor
    double svr_c;     // exp(-dt / tau)
};

// ---- launch wrappers (re_kernels.hip) -------------------------------------
// Each launches on `st` and returns the launch's hipError_t.
enum StepMode { kFused = 0, kStop = 1, kStopEnergy = 2, kQuery = 3, kRefresh = 4 };

hipError_t launch_start(bool fp64, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st);
// List update of the replicas [sa.r0, sa.r0 + nrep) whose update flag of
// parity sa.par is set (all with sa.force_all): work table, reorder by cell
// (one workgroup per replica, or grid-wide passes when `wide`), list build
// over the rebuilt replicas' atoms only.  atoms: sum of N over the range.
hipError_t launch_rebuild(bool fp64, const DevState& d, const StepArgs& sa, int nrep, int64_t atoms, bool wide,
                          hipStream_t st);
hipError_t launch_force(bool fp64, StepMode mode, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st);
hipError_t launch_energy(bool fp64, const DevState& d, const StepArgs& sa, int nrep, hipStream_t st);
hipError_t launch_exchange(const DevState& d, int R, int64_t attempt, uint64_t seed, double c1sq, int32_t master,
                           int64_t log_cap, int64_t step_all, int max_distance, hipStream_t st);
hipError_t launch_set_steps(const DevState& d, int R, int64_t step, hipStream_t st);
hipError_t launch_test_exchange(const double* U, const double* Tl, int32_t* slot, int R, uint64_t seed,
                                int64_t attempt, int max_distance, uint8_t* dec, hipStream_t st);
hipError_t launch_test_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, int n, uint32_t* out,
                              hipStream_t st);
hipError_t launch_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out, hipStream_t st);

// Record the message of a failed context-free call (re_last_error(NULL))
// and return code (re_host.cpp).
int fail_noctx(int code, const char* fmt, ...);

}  // namespace re
