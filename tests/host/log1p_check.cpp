// Host check of kbc::log1p_series (the logarithm of the exact stabilizer's
// root iteration) against the C library's log1pl in extended precision, over
// a dense grid of |x| < 1/16, near zero and at the ends; prints the largest
// relative error and fails above the bound given on the command line.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "kbc_device.h"

int main(int argc, char** argv)
{
    const double bound = argc > 1 ? std::atof(argv[1]) : 5e-16;
    double worst = 0.0, at = 0.0;
    auto check = [&](double x) {
        if (!kbc::log1p_series_ok(x) || x == 0.0) return;
        const long double ref = log1pl((long double)x);
        const double rel = (double)fabsl(((long double)kbc::log1p_series(x) - ref) / ref);
        if (rel > worst) { worst = rel; at = x; }
    };
    const int n = 2000000;
    for (int k = -n; k <= n; ++k) check(0.0625 * k / (n + 1.0));
    for (double x = 1e-300; x < 0.0625; x *= 1.37) { check(x); check(-x); }
    check(std::nextafter(0.0625, 0.0));
    check(-std::nextafter(0.0625, 0.0));
    std::printf("max relative error %.3e at x = %.17g\n", worst, at);
    return worst <= bound ? 0 : 1;
}
