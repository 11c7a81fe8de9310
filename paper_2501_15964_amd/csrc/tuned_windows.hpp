// Window chunk (incidences per row group of a window) for each row layout
// and q, as picked by the project's window tuner (tune_windows.py in the
// package: it times the Newton matvec over a sweep of chunks on synthetic
// k-NN graphs and rewrites this table).  Rows: the row layouts of
// dispatch_row in order (d <= 2, 4, 8, 16, 32, 64, 128, 256, 512, 768, 832,
// 1024); columns: q = 1, 2, inf.
#pragma once

namespace ccm {

constexpr int kTunedLayouts = 12;
constexpr int kTunedChunk[kTunedLayouts][3] = {
    {4, 4, 2}, {2, 2, 2}, {4, 4, 4}, {8, 8, 8},
    {16, 16, 16}, {32, 16, 32}, {32, 32, 64}, {32, 64, 128},
    {16, 64, 64}, {16, 32, 64}, {16, 64, 64}, {16, 32, 64},
};

}  // namespace ccm
