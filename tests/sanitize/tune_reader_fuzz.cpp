// Mutation fuzz of the tuning-file reader (host code only): argv[1] is a
// valid tuning file, argv[2] the number of mutated copies fed to
// lhs_tune_load and lhs_tune_lookup; for an AddressSanitizer and
// UndefinedBehaviorSanitizer build.  argv[3] is a scratch file path.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include "lhs.h"

static std::string slurp(const char *p) {
    FILE *f = fopen(p, "rb"); std::string s; char b[4096]; size_t n;
    while ((n = fread(b, 1, sizeof b, f)) > 0) s.append(b, n);
    fclose(f); return s;
}

int main(int argc, char **argv) {
    const std::string seed = slurp(argv[1]);
    const int iters = atoi(argv[2]);
    std::mt19937_64 rng(12345);
    const char *path = argv[3];
    const char alphabet[] = "{}[]\",:0123456789.eE+-truefalsnul\\u \n\t\"abcdefXYZ";
    int ok = 0, bad = 0;
    for (int it = 0; it < iters; ++it) {
        std::string s = seed;
        const int nm = 1 + rng() % 8;
        for (int k = 0; k < nm; ++k) {
            const int op = rng() % 5;
            const size_t pos = s.empty() ? 0 : rng() % s.size();
            if (op == 0 && !s.empty()) s.erase(pos, 1 + rng() % 16);
            else if (op == 1) s.insert(pos, 1, alphabet[rng() % (sizeof alphabet - 1)]);
            else if (op == 2 && !s.empty()) s[pos] = (char)(rng() & 0xFF);
            else if (op == 3) s.resize(rng() % (s.size() + 1));
            else if (op == 4) { std::string d(1 + rng() % 80, '['); s.insert(pos, d); }
        }
        FILE *f = fopen(path, "wb"); fwrite(s.data(), 1, s.size(), f); fclose(f);
        uint32_t n = 0;
        const lhs_status rc = lhs_tune_load(path, "gfx950", &n);
        (rc == LHS_OK ? ok : bad)++;
        lhs_config c; int32_t found;
        for (uint32_t W = 1; W <= 32; W += 7)
            lhs_tune_lookup(LHS_TUNE_TABLE, W, 1ull << (rng() % 33), &c, &found);
    }
    printf("iterations %d ok %d rejected %d\n", iters, ok, bad);
    return 0;
}
