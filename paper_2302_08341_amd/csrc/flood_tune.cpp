// Geometry defaults and the measured-choice cache of libflood.
//
// Cache file: $FLOOD_TUNE_CACHE (no caching when unset).  One line per tuned
// problem: "<key> mi tile_rows cpb".  Set FLOOD_AUTOTUNE=0 to skip measuring
// and use the defaults (or the explicit values given at creation).
#include "flood_tune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

namespace flood {

static std::string key_string(const TuneKey& k, int mi) {
    std::string s = "b" + std::to_string(k.real_bytes) + "_mi" + std::to_string(mi);
    for (int i = 0; i < k.n_catch; ++i)
        s += "_" + std::to_string(k.ny[i]) + "x" + std::to_string(k.nx[i]) + "x" + std::to_string(k.members[i]);
    return s;
}

TuneChoice tune_default(const TuneKey& k) {
    TuneChoice c;
    c.mi = 1;
    c.tile_rows = 4;
    int maxm = 1;
    for (int i = 0; i < k.n_catch; ++i) maxm = k.members[i] > maxm ? k.members[i] : maxm;
    c.cpb = maxm < 16 ? maxm : 16;
    return c;
}

bool tune_enabled() {
    const char* e = std::getenv("FLOOD_AUTOTUNE");
    return !(e && e[0] == '0');
}

bool tune_lookup(const TuneKey& k, int mi, TuneChoice& out) {
    const char* path = std::getenv("FLOOD_TUNE_CACHE");
    if (!path || !path[0]) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string want = key_string(k, mi);
    char key[512];
    int a, b, c;
    bool found = false;
    while (std::fscanf(f, "%511s %d %d %d", key, &a, &b, &c) == 4) {
        if (want == key) {
            out.mi = a;
            out.tile_rows = b;
            out.cpb = c;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const TuneKey& k, const TuneChoice& c) {
    const char* path = std::getenv("FLOOD_TUNE_CACHE");
    if (!path || !path[0]) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d\n", key_string(k, c.mi).c_str(), c.mi, c.tile_rows, c.cpb);
    std::fclose(f);
}

}  // namespace flood
