// re_tune.hpp -- autotuner interface (re_tune.cpp).
#pragma once
#include <cstdint>
#include <string>

#include "../../include/re.h"

namespace re {

constexpr int kTuneClasses = 32;  // size classes: floor(log2 N)

struct TuneChoice {
    int engine = -1;               // RE_LOCKSTEP | RE_PERSISTENT
    int tpa = 0;                   // force-kernel lanes per atom (every class without its own)
    int block = 0;                 // lockstep: threads per block of the wide kernels (0: default)
    double ms = 1e300;             // measured milliseconds per step
    int cls_tpa[kTuneClasses] = {};  // per size class: lanes per atom (0: tpa)
};

// The size class of a replica of N atoms: floor(log2 N).
int tune_class(int32_t N);

std::string tune_key(int R, const int32_t* N, const double* rho_r, double rho, double rc, double skin, int prec,
                     int xmode, int thermo);
bool tune_lookup(const char* path, const std::string& key, TuneChoice& out);
void tune_store(const char* path, const std::string& key, const TuneChoice& c);
int tune_run(int R, const int32_t* N, const double* T, double rho, double rc, double skin, double dt, int Nx,
             uint64_t seed, const re_options& base, TuneChoice& best);

}  // namespace re
