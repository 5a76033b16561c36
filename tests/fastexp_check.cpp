// Host build of the device exp/expm1 core: prints x, e^x, e^x - 1 in hex for
// the arguments read from stdin (one per line).
#include <cstdio>

#include "../paper_1901_07454_amd/csrc/fastexp.hpp"

int main() {
    double x;
    while (std::scanf("%la", &x) == 1) {
        const arbmi::ExpPair p = arbmi::exp_pair(x);
        std::printf("%a %a %a\n", x, p.e, p.em1);
    }
    return 0;
}
