// Host-only driver of the structure builder (structures.cpp) for the
// sanitizer test: builds every box given on the command line with the pure
// HP table and with Table 1 (x10), and prints the counts the Python side
// compares with the oracle.  Compiled with g++ and -fsanitize=address,undefined
// by tests/test_host_sanitizers.py; no GPU code is involved.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "hp_internal.h"

int main(int argc, char **argv)
{
    const int32_t tables[2][4] = {{0, 0, 0, -1}, {0, -10, -10, -23}};
    for (int a = 1; a + 2 < argc; a += 3) {
        const int X = std::atoi(argv[a]), Y = std::atoi(argv[a + 1]), Z = std::atoi(argv[a + 2]);
        for (int t = 0; t < 2; ++t) {
            hp_structs s;
            std::string msg;
            const hp_status st = hpmap::build_structures(X, Y, Z, tables[t], &s, &msg);
            std::printf("%d %d %d table %d status %d n_conf %u n_class %u nbp %u K %u K_pad %u "
                        "blk %d wide %d wide_s2 %zu\n",
                        X, Y, Z, t, int(st), s.n_conf, s.n_class, s.nbp, s.K, s.K_pad,
                        int(s.blk_ok), int(s.wide_ok), s.wide_s2.size());
        }
    }
    // argument errors are reported, not crashed on
    hp_structs bad;
    std::string msg;
    std::printf("bad %d\n", int(hpmap::build_structures(0, 3, 1, tables[0], &bad, &msg)));
    return 0;
}
