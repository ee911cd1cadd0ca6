// re_persist.hpp -- device state and launch interface of the persistent
// engine (re_persist.hip), shared with the host runtime.
#pragma once
#include "re_internal.hpp"

namespace re {

constexpr int kModeSync = 0, kModeAsync = 1, kModeSchedule = 2;
constexpr unsigned kErrTimeout = 1u;

// Device state of the exchange protocol and of the replicas' progress
// (persists across calls unless noted).
struct PersistState {
    int32_t* slotbuf;   // 2 x R: slot held entering an attempt of parity p
    int64_t* post;      // R: last posted attempt + 1 (mailbox flag)
    double* upost;      // 2 x R: posted energies, by attempt parity
    int64_t* spost;     // 2 x R: posted join steps
    int32_t* apend;     // R: velocity factor pending for the next step
    int64_t* katt;      // R: next attempt index of each replica
    int64_t* jprev;     // R: step of each replica's last exchange join
    int32_t* ctl;       // 2 x R: leader -> team control words (per call)
    uint64_t* xdone;    // resolutions in this call (reset per call)
    uint64_t* trig;     // next attempt to be triggered (asynchronous mode)
    uint32_t* parked;   // replicas parked at the end of the call (per call)
    uint32_t* reach;    // asynchronous mode: replicas that reached their target (per call)
    uint64_t* beat;     // progress heartbeat: force phases completed
    uint32_t* abort;    // nonzero: every team leaves
    uint32_t* err;      // kErr* bits
    uint32_t* xmask;    // per team: XCDs its workgroups run on (per call)
};

// Per-call parameters, in device memory (updated before each launch).
struct CallParams {
    int mode;             // kModeSync | kModeAsync | kModeSchedule
    int cur0;             // position buffer holding the current positions
    int apply_alpha;      // nonzero: every replica's pending velocity factor (set
                          // outside the engine, e.g. by re_exchange) is applied by
                          // its first step
    int64_t k0;           // first attempt index of the call
    int64_t n;            // sync/async: steps each replica advances (its target is
                          // its step count at the call's start plus n)
    const int64_t* sched; // A x R join steps (schedule mode)
    int64_t A;
};

struct PersistArgs {
    StepArgs sa;              // h, c1, u(r_c), seed, R, tpa, M
    PersistState st;
    const CallParams* call;
    const int32_t* team_rep;  // per block: replica (-1: idle)
    const int32_t* team_mem;  // per block: member index within the team
    const int32_t* team_size; // per block: team size
    const int32_t* team_id;   // per block: team index (barrier counter)
    unsigned* bar;            // 64 counters per team (one cache line each)
    int Nx;
    double c1sq;
    int64_t log_cap;
    uint64_t timeout;         // watchdog, in 100 MHz clock ticks without progress
    int xmaxd;                // largest ladder distance of an exchange pair (1: nearest neighbours)
    int bar_mode;             // team barrier: 0 agent-scope release + acquire; 1 for teams on one
                              // XCD: stores complete to the shared L2 + agent-scope acquire
    uint32_t delay_ticks;     // test hook: pauses after team barriers, in 100 MHz ticks (0: off)
};

hipError_t launch_persist(bool fp64, const DevState& d, const PersistArgs& pa, int nblk, int nteams, hipStream_t st);
hipError_t persist_occupancy(bool fp64, bool n16, int tpa, bool svr, int* blocks_per_cu);

}  // namespace re
