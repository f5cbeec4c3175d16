// opcount.cpp -- instrumented build of the CPU oracle that counts the
// floating-point operations of each ray, by category.
//
// TEST INFRASTRUCTURE ONLY (like ray_oracle.c, which it compiles unchanged):
// only tests/ and the benchmark's documentation of its FLOP constants use it.
//
// The oracle's source is compiled as C++ with every `double` replaced by a
// value type that counts its arithmetic: +, -, *, / and each call of sqrt,
// exp, log, sin, cos, pow, cbrt, log1p, expm1 or fmod is one operation;
// comparisons, fabs, floor, negation and conversions are free.  The oracle
// marks its categories with OR_CAT: 0 = geodesic (right-hand sides, RK4
// combination, step rule, midpoint, features), 1 = plasma point (flow, field,
// frame, polarisation angle, coefficients), 2 = transfer update.
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

namespace opc {
thread_local long long n[4];   // operations per category
thread_local int cat;          // current category
thread_local long long emit;   // steps whose plasma point emits
thread_local long long noemit; // plasma-point operations of the other steps
thread_local long long before; // category-1 count when the plasma point began
inline void tick() { ++n[cat]; }
}  // namespace opc

struct cd {
    double v;
    cd() = default;
    cd(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator float() const { return (float)v; }
    explicit operator int() const { return (int)v; }
    explicit operator long long() const { return (long long)v; }
    cd& operator+=(cd o) { opc::tick(); v += o.v; return *this; }
    cd& operator-=(cd o) { opc::tick(); v -= o.v; return *this; }
    cd& operator*=(cd o) { opc::tick(); v *= o.v; return *this; }
    cd& operator/=(cd o) { opc::tick(); v /= o.v; return *this; }
};
inline cd operator+(cd a, cd b) { opc::tick(); return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { opc::tick(); return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { opc::tick(); return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { opc::tick(); return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }
inline bool operator<(cd a, cd b) { return a.v < b.v; }
inline bool operator>(cd a, cd b) { return a.v > b.v; }
inline bool operator<=(cd a, cd b) { return a.v <= b.v; }
inline bool operator>=(cd a, cd b) { return a.v >= b.v; }
inline bool operator==(cd a, cd b) { return a.v == b.v; }
inline bool operator!=(cd a, cd b) { return a.v != b.v; }
#define OPC_F1(f) inline cd f(cd a) { opc::tick(); return cd(::f(a.v)); }
OPC_F1(sqrt) OPC_F1(exp) OPC_F1(log) OPC_F1(sin) OPC_F1(cos) OPC_F1(cbrt) OPC_F1(log1p) OPC_F1(expm1)
#undef OPC_F1
inline cd pow(cd a, cd b) { opc::tick(); return cd(::pow(a.v, b.v)); }
inline cd fmod(cd a, cd b) { opc::tick(); return cd(::fmod(a.v, b.v)); }
inline cd fabs(cd a) { return cd(::fabs(a.v)); }
inline cd floor(cd a) { return cd(::floor(a.v)); }

#define OR_CAT(c) (opc::cat = (c), (c) == 1 ? (void)(opc::before = opc::n[1]) : (void)0)
#define OR_EMIT(e) ((e) ? (void)++opc::emit : (void)(opc::noemit += opc::n[1] - opc::before))
#define double cd
extern "C" {
#include "ray_oracle.c"
}
#undef double

// Trace one ray with counting: out[0] steps, out[1] emitting steps, out[2..4]
// operations of categories 0..2, out[5] plasma-point operations of the
// steps that do not emit (inside category 1); S[0..3] the ray's Stokes
// values (the same computation as the plain build's).
extern "C" int or_count_ray(const or_params* p, double al, double be, long long* out, double* S_out)
{
    for (int k = 0; k < 4; ++k) opc::n[k] = 0;
    opc::cat = 0;
    opc::emit = opc::noemit = 0;
    cd S[4 + OR_MAX_SUB];
    ray_feat ft;
    trace_one(p, cd(al), cd(be), S, &ft, 0, 0, 0);
    out[0] = ft.steps;
    out[1] = opc::emit;
    out[2] = opc::n[0];
    out[3] = opc::n[1];
    out[4] = opc::n[2];
    out[5] = opc::noemit;
    for (int k = 0; k < 4; ++k) S_out[k] = (double)S[k];
    return ft.status;
}

// Operations of single oracle routines, for pinning the counter itself:
// which = 0: one 4x4 matrix product; 1: the horizon radius.
extern "C" long long or_count_probe(int which)
{
    for (int k = 0; k < 4; ++k) opc::n[k] = 0;
    opc::cat = 0;
    if (which == 0) {
        cd A[16], B[16], C[16];
        for (int i = 0; i < 16; ++i) { A[i] = cd(0.5 + i); B[i] = cd(1.0 - 0.25 * i); }
        matmul4(A, B, C);
    } else {
        volatile double r = (double)horizon(cd(0.5));
        (void)r;
    }
    return opc::n[0];
}
