// The description of a spline's generated tables that the host library works
// from (lattice, cosets, directions, stencil extent), filled from the tables
// of one kind.  The library fills it for its built-in splines; a spline
// compiled at run time into its own shared library (a plugin) fills it for
// its tables and exports
//
//   extern "C" int lsp_plugin_describe(lsp::SplineDesc* d);     // 0 on success
//   extern "C" hipError_t lsp_plugin_eval(const lsp::EvalArgs* a);
//
// built from the same headers, so both sides agree on these structs; the ABI
// number below changes whenever either layout does.
#pragma once

#include "lsp_launch.h"
#include "lsp_locate.h"

namespace lsp {

constexpr int kDescMaxDirs = 16;
struct SplineDesc;

struct SplineDesc {
    int abi;
    int kind;
    char name[32];
    int lattice;                   // 0 Z^3, 1 BCC, 2 FCC
    int symmetry;                  // Sym
    int L[3][3];                   // columns are generators
    int n_dirs;
    int dirs[kDescMaxDirs][3];     // with repeats
    int n_cosets, D, shift[4][3];
    int taps, union_taps, n_reference, degree, radius, fma_eval;
    int off_lo, off_hi;            // min / max stencil offset component (reference frame)
};

// version 1; the struct sizes catch a layout change made without a new version
constexpr int kPluginAbi = (1 << 24) | ((int)sizeof(EvalArgs) << 12) | (int)sizeof(SplineDesc);

template <int K>
void describe(SplineDesc* d) {
    using T = TablesOf<K>;
    *d = SplineDesc{};
    d->abi = kPluginAbi;
    d->kind = K;
    const char* nm = gen::SplineOf<K>::kName;
    for (int i = 0; i < 31 && nm[i]; ++i) d->name[i] = nm[i];
    d->lattice = T::kLattice;
    d->symmetry = T::kSymmetry;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) d->L[i][j] = T::kL[i][j];
    static_assert(T::kNumDirs <= kDescMaxDirs, "too many directions for the description");
    d->n_dirs = T::kNumDirs;
    for (int k = 0; k < T::kNumDirs; ++k)
        for (int a = 0; a < 3; ++a) d->dirs[k][a] = T::kXi[k][a];
    d->n_cosets = T::kNumCosets;
    d->D = T::kD;
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 3; ++a) d->shift[m][a] = T::kShift[m][a];
    d->taps = __builtin_popcountll(T::kRegionMask0);
    d->union_taps = T::kTaps;
    d->n_reference = T::kRegions;
    d->degree = T::kDegree;
    d->radius = T::kRadius;
    d->fma_eval = T::kFmaEval;
    int lo = 0, hi = 0;
    for (int j = 0; j < T::kTaps; ++j)
        for (int a = 0; a < 3; ++a) {
            lo = T::kOff[j][a] < lo ? T::kOff[j][a] : lo;
            hi = T::kOff[j][a] > hi ? T::kOff[j][a] : hi;
        }
    d->off_lo = lo;
    d->off_hi = hi;
}

}  // namespace lsp
