// Host-side evaluation of the solver's erfc approximation on arguments read
// from stdin (one per line); prints erfc in FP64 and FP32 paths.  The
// reciprocal 1/(c + |y|) is formed here by division (the kernels refine the
// hardware estimate to within an ulp or two of it).  With the argument
// "exp" it prints the solver's exponential of each input instead.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../paper_2108_07031_amd/csrc/qlskum_erfc.h"

int main(int argc, char **argv) {
    const bool exp_mode = argc > 1 && std::strcmp(argv[1], "exp") == 0;
    double y;
    while (std::scanf("%lf", &y) == 1) {
        if (exp_mode) {
            std::printf("%.17e\n", ql::exp_poly(y));
            continue;
        }
        const double e64 =
            2.0 * ql::half_erfc(y, ql::gauss(y), 1.0 / (ql::kErfcC64 + std::fabs(y)));
        const float yf = (float)y;
        const float e32 = 2.0f * ql::half_erfc_f(yf, std::exp(-yf * yf),
                                                 1.0f / (ql::kErfcC32 + std::fabs(yf)));
        std::printf("%.17e %.9e\n", e64, (double)e32);
    }
    return 0;
}
