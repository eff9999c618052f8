// gd_twiddle.h -- compile-time table of FFT twiddle factors.
//
// kTw[k] = (cos(2 pi k / kTwN), -sin(2 pi k / kTwN)) = exp(-2 pi i k / kTwN),
// k < kTwN / 2, in FP64.  A transform of length n <= kTwN uses the entries at
// stride kTwN / n.  The table is evaluated by the compiler from Taylor series
// on [0, pi/4], with the exact integer reduction k -> (quadrant, octant), so it
// needs no initialisation at run time.  Plain C++: tests/test_twiddle_table.py
// compiles it with the host compiler and checks it against the C library's
// sin and cos.
#pragma once

namespace gdtw {

constexpr int kTwLog = 12;
constexpr int kTwN = 1 << kTwLog;  // longest transform: 4096 points

struct Cd {
    double re, im;
};

// sin and cos of x for |x| <= pi/4: the series terms fall below 1e-17 after
// 12 terms; 24 are taken.
constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 24; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 24; ++n) {
        term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}

constexpr double kPi = 3.14159265358979323846264338327950288;

// exp(-2 pi i k / kTwN) for 0 <= k < kTwN / 2.
constexpr Cd twiddle(int k) {
    const int q = k / (kTwN / 4);            // quadrant: angle = q pi/2 + t
    const int r = k % (kTwN / 4);            // t = 2 pi r / kTwN in [0, pi/2)
    double c, s;                             // cos t, sin t
    if (r <= kTwN / 8) {
        const double t = 2.0 * kPi * r / kTwN;
        c = taylor_cos(t);
        s = taylor_sin(t);
    } else {                                 // t > pi/4: use pi/2 - t
        const double t = 2.0 * kPi * (kTwN / 4 - r) / kTwN;
        c = taylor_sin(t);
        s = taylor_cos(t);
    }
    // rotate by q quarter turns: (c, s) -> (-s, c)
    for (int i = 0; i < q; ++i) {
        const double tmp = c;
        c = -s;
        s = tmp;
    }
    return Cd{c, -s};
}

struct Table {
    Cd v[kTwN / 2];
};

constexpr Table make_table() {
    Table t{};
    for (int k = 0; k < kTwN / 2; ++k) t.v[k] = twiddle(k);
    return t;
}

}  // namespace gdtw
