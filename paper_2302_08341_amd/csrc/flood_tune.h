// Kernel-geometry tuner of libflood: the key of a tuning problem, the chosen
// geometry, the defaults used before (or instead of) measuring, and a small
// text cache of measured choices.
#pragma once

namespace flood {

struct TuneKey {
    int real_bytes;
    int n_catch;
    int ny[8], nx[8], members[8];
};

struct TuneChoice {
    int mi = 1;          // members interleaved in the fastest index
    int tile_rows = 4;   // cell rows per 256-lane tile
    int cpb = 16;        // member chunks per workgroup
    int variant = 1;     // 1 tiled kernel, 2 row-marching kernel
    int march_rows = 32; // rows per strip of the row-marching kernel
    int march_seg = 2;   // members marched together by one wavefront
    int march_order = 1; // wavefront order of the row-march kernels (0 to 4)
    int march_rows_c[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // per catchment, 0: march_rows
};

TuneChoice tune_default(const TuneKey& k);
bool tune_enabled();
bool tune_lookup(const TuneKey& k, int mi, TuneChoice& out);
void tune_store(const TuneKey& k, const TuneChoice& c);

}  // namespace flood
