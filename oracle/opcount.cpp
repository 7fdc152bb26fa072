// Operation-counting build of the CPU oracle (test infrastructure).
//
// Compiles hydro_oracle.c unchanged with `double` replaced by a counting
// type, so every floating-point operation the oracle performs is tallied:
// add, subtract, multiply, divide, square root and power as flops, and
// comparisons separately.  Negation, |x| and copysign are sign manipulations
// and are not counted.  Literal constant expressions (1.0/6.0, ...) fold at
// compile time and are not counted either.
//
// opcount_* entry points return the counts of one call of the corresponding
// oracle routine so a harness can split the work by step of the method.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace {
uint64_t g_flop = 0;
uint64_t g_cmp = 0;
}  // namespace

struct cd {
    double v;
    cd() = default;
    constexpr cd(double x) : v(x) {}
    constexpr cd(int x) : v((double)x) {}
    constexpr cd(long x) : v((double)x) {}
};
inline cd operator+(cd a, cd b) { ++g_flop; return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { ++g_flop; return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { ++g_flop; return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { ++g_flop; return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }
inline bool operator<(cd a, cd b) { ++g_cmp; return a.v < b.v; }
inline bool operator>(cd a, cd b) { ++g_cmp; return a.v > b.v; }
inline bool operator<=(cd a, cd b) { ++g_cmp; return a.v <= b.v; }
inline bool operator>=(cd a, cd b) { ++g_cmp; return a.v >= b.v; }
inline cd fabs(cd a) { return cd(std::fabs(a.v)); }
inline cd copysign(cd a, cd b) { return cd(std::copysign(a.v, b.v)); }
inline cd sqrt(cd a) { ++g_flop; return cd(std::sqrt(a.v)); }
inline cd pow(cd a, cd b) { ++g_flop; return cd(std::pow(a.v, b.v)); }
// a classification, not arithmetic: not counted
inline bool isnan(cd a) { return std::isnan(a.v); }

#define double cd
#include "hydro_oracle.c"
#undef double

extern "C" {

void opcount_reset(void) { g_flop = 0; g_cmp = 0; }
void opcount_read(uint64_t *flop, uint64_t *cmp) { *flop = g_flop; *cmp = g_cmp; }

// Counting versions of the oracle entry points on plain double buffers.
void opcount_ppm(const double *q5, double *lr) {
    cd q[5];
    for (int i = 0; i < 5; ++i) q[i] = cd(q5[i]);
    cd L, R;
    oracle_ppm(q, &L, &R);
    lr[0] = L.v;
    lr[1] = R.v;
}

double opcount_point_flux(int n, const double *ul, const double *ur, const double *x,
                          double gamma, double omega, double eta1, double *F) {
    cd UL[7], UR[7], xq[3], Fc[7];
    for (int f = 0; f < 7; ++f) { UL[f] = cd(ul[f]); UR[f] = cd(ur[f]); }
    for (int a = 0; a < 3; ++a) xq[a] = cd(x[a]);
    oracle_phys ph;
    ph.gamma = cd(gamma);
    ph.omega = cd(omega);
    ph.eta1 = cd(eta1);
    ph.eta2 = cd(0.1);
    ph.centre_only = 0;
    ph.reflux = 0;
    cd a = oracle_point_flux(n, UL, UR, xq, &ph, Fc);
    for (int f = 0; f < 7; ++f) F[f] = Fc[f].v;
    return a.v;
}

// L(U) of one padded block (flux divergence, source), the new scheme or (with
// centre_only) the old face-centre one; the counts include the oracle's
// reconstruction of all 13 lines at every cell -1..8 per axis.
void opcount_leaf_rhs(const double *P, double dx, const double *origin, double gamma,
                      double omega, double eta1, int centre_only, double *dU) {
    const long np = 7L * 2744;
    cd *Pc = (cd *)malloc(sizeof(cd) * np);
    cd *dUc = (cd *)malloc(sizeof(cd) * 7 * 512);
    for (long i = 0; i < np; ++i) Pc[i] = cd(P[i]);
    cd org[3] = {cd(origin[0]), cd(origin[1]), cd(origin[2])};
    oracle_phys ph;
    ph.gamma = cd(gamma);
    ph.omega = cd(omega);
    ph.eta1 = cd(eta1);
    ph.eta2 = cd(0.1);
    ph.centre_only = centre_only;
    ph.reflux = 0;
    cd am;
    oracle_leaf_rhs(Pc, cd(dx), org, &ph, dUc, &am);
    for (int i = 0; i < 7 * 512; ++i) dU[i] = dUc[i].v;
    free(dUc);
    free(Pc);
}

}  // extern "C"
