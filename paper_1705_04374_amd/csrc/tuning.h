// Tile / schedule choice of the stage kernel per (precision, dimension, size).
// Defaults are set here; ofm_tune_set overrides one entry and ofm_autotune
// measures the compiled candidates and stores the fastest.
#pragma once

#include <map>
#include <tuple>

namespace ofm {

struct TileChoice {
    int tx, ty, zchunk, graph_steps;
};

struct Tuning {
    // key: (precision, ndim, size class = ceil(log2 n)); the WENO order and
    // the boundary condition share an entry (the last autotune wins)
    std::map<std::tuple<int, int, int>, TileChoice> table;

    static int size_class(int n)
    {
        int c = 0;
        while ((1 << c) < n) ++c;
        return c;
    }

    TileChoice choose(int precision, int ndim, int maxn, int /*n_samples*/) const
    {
        auto it = table.find(std::make_tuple(precision, ndim, size_class(maxn)));
        if (it != table.end()) return it->second;
        TileChoice t;
        if (ndim == 3) {
            // the autotuner's picks on the 500-bubble cloud: float 16 x 16
            // tiles of 16 planes up to 256^3, double 16 x 14 tiles of 16
            // planes; both 16 x 14 tiles of 32 planes at 512^3 and above
            t.tx = 16;
            t.ty = precision == 1 || maxn >= 512 ? 14 : 16;
            t.zchunk = maxn >= 512 ? 32 : 16;
        } else if (ndim == 2) {
            t.tx = 16;
            t.ty = 14;
            t.zchunk = 1;
        } else {
            t.tx = 256;
            t.ty = 1;
            t.zchunk = 1;
        }
        t.graph_steps = maxn >= 256 ? 4 : 16;
        return t;
    }

    void set(int precision, int ndim, int n, const TileChoice& t)
    {
        table[std::make_tuple(precision, ndim, size_class(n))] = t;
    }
};

}  // namespace ofm
