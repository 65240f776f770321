// Geometry defaults and the measured-choice cache of libflood.
//
// Measured choices are remembered for the life of the process, so handles of
// one problem shape after the first do not measure again, and optionally in a
// file: $FLOOD_TUNE_CACHE, one line per tuned problem,
// "<key> mi tile_rows cpb variant march_rows march_seg march_order rows_1,...,rows_n"
// (the last field: each catchment's rows per strip, 0 for march_rows).  Set
// FLOOD_AUTOTUNE=0 to skip measuring and use the defaults (or the explicit
// values given at creation).
#include "flood_tune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
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
    c.variant = 3;      // vectorised row march (falls back to 2 when nx does not allow it)
    c.march_rows = 16;
    c.march_seg = 1;
    c.march_order = 1;
    return c;
}

bool tune_enabled() {
    const char* e = std::getenv("FLOOD_AUTOTUNE");
    return !(e && e[0] == '0');
}

static std::mutex memo_mu;
static std::map<std::string, TuneChoice>& memo() {
    static std::map<std::string, TuneChoice> m;
    return m;
}

bool tune_lookup(const TuneKey& k, int mi, TuneChoice& out) {
    {
        std::lock_guard<std::mutex> lock(memo_mu);
        auto it = memo().find(key_string(k, mi));
        if (it != memo().end()) {
            out = it->second;
            return true;
        }
    }
    const char* path = std::getenv("FLOOD_TUNE_CACHE");
    if (!path || !path[0]) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string want = key_string(k, mi);
    char line[1024], key[512], rows[256];
    int a, b, c, d, e, f2, g2;
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        rows[0] = 0;
        const int got = std::sscanf(line, "%511s %d %d %d %d %d %d %d %255s", key, &a, &b, &c, &d, &e, &f2, &g2, rows);
        if (got < 8) continue;
        // an entry outside the geometries this library launches is ignored
        bool sane = (a == 1 || a == 2 || a == 4 || a == 8) && b >= 1 && b <= 8 && c >= 1 && d >= 1 && d <= 3 &&
                    e >= 1 && e <= 4096 && (f2 == 1 || f2 == 2 || f2 == 4 || f2 == 8) && g2 >= 0 && g2 <= 4;
        int rc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (got == 9) {
            const char* p = rows;
            for (int i = 0; i < k.n_catch && i < 8 && *p; ++i) {
                char* end = nullptr;
                const long v = std::strtol(p, &end, 10);
                if (end == p || v < 0 || v > 4096) { sane = false; break; }
                rc[i] = (int)v;
                p = *end == ',' ? end + 1 : end;
            }
        }
        if (want == key && sane) {
            out.mi = a;
            out.tile_rows = b;
            out.cpb = c;
            out.variant = d;
            out.march_rows = e;
            out.march_seg = f2;
            out.march_order = g2;
            for (int i = 0; i < 8; ++i) out.march_rows_c[i] = rc[i];
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const TuneKey& k, const TuneChoice& c) {
    {
        std::lock_guard<std::mutex> lock(memo_mu);
        memo()[key_string(k, c.mi)] = c;
    }
    const char* path = std::getenv("FLOOD_TUNE_CACHE");
    if (!path || !path[0]) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::string rows;
    for (int i = 0; i < k.n_catch && i < 8; ++i) rows += (i ? "," : "") + std::to_string(c.march_rows_c[i]);
    std::fprintf(f, "%s %d %d %d %d %d %d %d %s\n", key_string(k, c.mi).c_str(), c.mi, c.tile_rows, c.cpb, c.variant,
                 c.march_rows, c.march_seg, c.march_order, rows.c_str());
    std::fclose(f);
}

}  // namespace flood
