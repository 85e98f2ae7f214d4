// build_state.h -- temporaries shared by the build stages (build.hip,
// hilbert.hip).  Not part of the public ABI.
#pragma once

#include <algorithm>
#include <vector>

#include "sba_internal.h"

#define SC_SLOTS 32
#define SC_READ 20
// slot of the largest polygon's event count (read with the edge totals)
#define SC_SEG_MAX 14
// slot of the largest row's toggle count (read with the toggle total)
#define SC_ROW_MAX 15
// slots of the set table path: distinct sets, total member ids
#define SC_SET_N 18
#define SC_SET_IDS 19

struct BuildState {
    explicit BuildState(hipStream_t s) : st(s), ws(s) {}
    hipStream_t st;
    Workspace ws;  // temporaries; returned (after a sync) when the build ends

    template <typename T>
    int alloc(T **p, int64_t n)
    {
        return ws.alloc(p, n);
    }
    void release(void *p) { ws.put(p); }

    // device scalars of the build (error bits, sizes, scan totals) that are
    // read back together: slots [0, SC_READ) in one copy
    int64_t *sc = nullptr;

    bool boundary_only = false;  // no interior spans: B(P) only
    bool centre = false;         // centre-sampled cells: crossings of the centre lines only

    // clip window in coordinates, [wx0, wx1) x [wy0, wy1)
    bool window = false;
    int64_t wx0 = 0, wy0 = 0, wx1 = 0, wy1 = 0;
    bool empty = false;  // the window holds no cell of any polygon
    // Hilbert key grid given by the caller (key_level 0: the stored box's own)
    int32_t key_level = 0;
    int64_t key_i0 = 0, key_j0 = 0;
    // edges: (x1,y1,x2,y2) and polygon id, one per vertex
    int4 *edges = nullptr;
    int32_t *epoly = nullptr;
    int64_t n_edges = 0;
    int xbits = 0, rbits = 0;    // event key fields: row << xbits | x
    int64_t NB = 0;              // boundary intervals (events [0, 2 NB) until sorted)
    uint64_t *evkey = nullptr;
    uint32_t *evpay = nullptr;
    // row segments of constant polygon set
    int64_t NS = 0;
    int64_t *seg_row_off = nullptr;  // [gh+1]
    int32_t *seg_x0 = nullptr, *seg_x1 = nullptr;
    uint32_t *seg_code = nullptr;
    // Hilbert layout: unique keys of boundary cells
    int (*on_boundary_events)(BuildState &, sba_handle *, hipStream_t) = nullptr;
    uint64_t *bkeys = nullptr;
    int64_t nbkeys = 0;
};

int build_segments(const sba_polygons *polys, int64_t eps, hipStream_t st, sba_handle *h,
                   BuildState &B, bool need_boundary_cells);
int hilbert_prepare(BuildState &B, sba_handle *h);
int hilbert_finish(BuildState &B, sba_handle *h, const sba_build_opts &o, hipStream_t st);
