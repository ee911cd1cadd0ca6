// re_tune.hpp -- autotuner interface (re_tune.cpp).
#pragma once
#include <cstdint>
#include <string>

#include "../../include/re.h"

namespace re {

struct TuneChoice {
    int engine;  // RE_LOCKSTEP | RE_PERSISTENT
    int tpa;     // force-kernel lanes per atom
    double ms;   // measured milliseconds per step
};

std::string tune_key(int R, const int32_t* N, const double* rho_r, double rho, double rc, double skin, int prec,
                     int xmode, int thermo);
bool tune_lookup(const char* path, const std::string& key, TuneChoice& out);
void tune_store(const char* path, const std::string& key, const TuneChoice& c);
int tune_run(int R, const int32_t* N, const double* T, double rho, double rc, double skin, double dt, int Nx,
             uint64_t seed, const re_options& base, TuneChoice& best);

}  // namespace re
