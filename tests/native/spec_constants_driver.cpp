// Test driver: prints the library's host-side specification constants for the
// (seed, t) pairs given on the command line, one line per value, so that a
// test can build the constants code under AddressSanitizer and
// UndefinedBehaviorSanitizer and compare its output with the oracle's.
#include <cinttypes>
#include <cstdio>
#include <cstdlib>

#include "../../paper_2005_11547_amd/csrc/dms_internal.h"

int main(int argc, char** argv)
{
    for (int a = 1; a + 1 < argc; a += 2) {
        const uint64_t seed = std::strtoull(argv[a], nullptr, 10);
        const uint32_t t = (uint32_t)std::strtoul(argv[a + 1], nullptr, 10);
        static dms::SpecTables sp;
        if (!dms::make_spec(seed, t, &sp)) {
            std::printf("fail %" PRIu64 " %u\n", seed, t);
            return 1;
        }
        std::printf("keys %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 "\n",
                    sp.key_r, sp.key_a, sp.key_u, sp.key_v, sp.key_s, sp.key_l);
        std::printf("pois");
        for (int n = 0; n < dms::kNumPoisson; ++n) std::printf(" %" PRIu64, sp.pois[n]);
        std::printf("\nW");
        for (int i = 0; i < dms::kMaxIndex; ++i) std::printf(" %a", dms::corner_w(sp, i));
        std::printf("\nR");
        for (int i = 0; i < dms::kMaxIndex; ++i) std::printf(" %a", dms::corner_r(sp, i));
        std::printf("\nu %a\ntab", sp.u);
        for (int i = 0; i < dms::kTabWords; ++i) std::printf(" %" PRIu64, sp.tab[i]);
        std::printf("\n");
    }
    for (int k = 1; k <= 4096; ++k) std::printf("%u%c", dms::t_of_k(k), k == 4096 ? '\n' : ' ');
    return 0;
}
