// perm_plan.h -- host-side plan of the LDS-tiled permute (plain C++, no HIP).
//
// A permute out[i] = in[sum_k c_k is_k] (c = digits of i over the output dims
// od, row-major) that moves the input's contiguous axis away from the
// output's reads the input in short strided runs when done element by element.
// The tiled form splits the dims into
//   * a unit U: the trailing dims contiguous in both input and output,
//   * an in-block: the input's next contiguous dims (strides U, U d1, ...),
//   * an out-block: the output's next contiguous dims (from the end),
//   * the rest,
// and moves one tile (a chunk of the in-block x a chunk of the out-block x U)
// per workgroup through LDS: reads run along the in-block, writes along the
// out-block.  All offsets fit in 32 bits (the caller keeps n < 2^31).
#pragma once
#include <algorithm>
#include <cstdint>

namespace ctmk {

constexpr int kPermTileElems = 2048;   // doubles per tile (16 KiB of LDS)
constexpr int kPermTileSide = 256;     // largest chunk of either block
constexpr int kPermBlockDims = 4;
constexpr int64_t kPermShortRunElems = 1250000;   // size from which 4-element block runs are tiled
constexpr int kPermRestDims = 12;

// q = x / d for x < 2^31 as (umulhi(x, mul) + x) >> shr, with shr =
// ceil(log2 d) and mul = floor(2^32 (2^shr - d) / d) + 1
struct FastDiv {
    uint32_t d, mul, shr;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t sh = 0;
    while (((uint64_t)1 << sh) < d) ++sh;
    const uint64_t m = ((((uint64_t)1 << 32) * (((uint64_t)1 << sh) - d)) / d) + 1;
    return FastDiv{d, (uint32_t)m, sh};
}

struct PermTile {
    int U;                 // unit length
    int TI, TO;            // chunk lengths of the in- and out-block
    int Lin, Lout;         // in- and out-block lengths
    int nci, nco;          // chunks per block
    int nin, nout, nrest;
    int in_d[kPermBlockDims], in_os[kPermBlockDims];      // in-block dims (fastest first), output strides
    int out_d[kPermBlockDims], out_is[kPermBlockDims];    // out-block dims (fastest first), input strides
    int rest_is[kPermRestDims], rest_os[kPermRestDims];
    FastDiv rest_d[kPermRestDims];                        // rest dims
    FastDiv fU, fci, fco;                                 // U, nci, nco
    FastDiv frun[2], fruno[2];   // load / store row lengths TI U, TO U: full chunk, last chunk
    int64_t tiles;         // product of rest dims x nci x nco
};

// Plan the tiled form of a permute given by its output dims od[0..rank-1] and
// the input stride is[k] of each output dim, n = product of od < 2^31.
// Returns false where the element-wise kernel is as good (the unit is already
// a long contiguous run, or one of the blocks would be short).
inline bool plan_perm_tile(int rank, const int64_t* od, const int64_t* is, PermTile& t)
{
    struct Dim { int64_t d, is, os; };
    Dim v[kPermRestDims + 1];
    int r = 0;
    int64_t os = 1;
    int64_t ostride[kPermRestDims + 1];
    if (rank < 1 || rank > kPermRestDims) return false;
    for (int k = rank - 1; k >= 0; --k) { ostride[k] = os; os *= od[k]; }
    for (int k = 0; k < rank; ++k)
        if (od[k] > 1) v[r++] = Dim{od[k], is[k], ostride[k]};
    // merge output-adjacent dims that are adjacent in the input too
    int m = 0;
    for (int k = 0; k < r; ++k) {
        if (m > 0 && v[m - 1].is == v[k].is * v[k].d) {
            v[m - 1].d *= v[k].d;
            v[m - 1].is = v[k].is;
            v[m - 1].os = v[k].os;
        } else {
            v[m++] = v[k];
        }
    }
    r = m;
    if (r < 2) return false;
    int64_t U = 1;
    if (v[r - 1].is == 1) { U = v[r - 1].d; --r; }
    if (U >= 32 || r < 2) return false;
    const int64_t want = std::max<int64_t>(1, 64 / U);
    bool used[kPermRestDims + 1] = {};
    // in-block: dims with input strides U, U d1, U d1 d2, ...; its first dim
    // (input stride U) is never the output's fastest remaining one (the two
    // would have merged into the unit)
    t.nin = 0;
    int64_t Lin = 1;
    auto grow_in = [&]() {
        while (Lin < want && t.nin < kPermBlockDims) {
            int f = -1;
            for (int k = 0; k < r; ++k)
                if (v[k].is == U * Lin) { f = k; break; }
            if (f < 0 || used[f]) break;
            used[f] = true;
            t.in_d[t.nin] = (int)v[f].d;
            t.in_os[t.nin] = (int)v[f].os;
            ++t.nin;
            Lin *= v[f].d;
            if (t.nin == 1) break;
        }
    };
    grow_in();
    // out-block: trailing output dims (before the in-block takes more, so
    // that the output's run is not cut short)
    t.nout = 0;
    int64_t Lout = 1;
    for (int k = r - 1; k >= 0 && Lout < want && t.nout < kPermBlockDims; --k) {
        if (used[k]) break;
        used[k] = true;
        t.out_d[t.nout] = (int)v[k].d;
        t.out_is[t.nout] = (int)v[k].is;
        ++t.nout;
        Lout *= v[k].d;
    }
    grow_in();
    // shortest block run (elements) worth a tile: 8, and 4 for large permutes,
    // where a tile with 4-7 element rows (partial writes or reads of 32-56
    // bytes) still beats the element-wise kernel's strided reads (measured
    // from 1.25e6 elements up; below that the element-wise kernel is faster)
    const int64_t min_run = os >= kPermShortRunElems ? 4 : 8;
    if (t.nin == 0 || t.nout == 0 || Lin * U < min_run || Lout * U < min_run) return false;
    t.nrest = 0;
    int64_t rest = 1;
    for (int k = 0; k < r; ++k) {
        if (used[k]) continue;
        t.rest_d[t.nrest] = make_fastdiv((uint32_t)v[k].d);
        t.rest_is[t.nrest] = (int)v[k].is;
        t.rest_os[t.nrest] = (int)v[k].os;
        ++t.nrest;
        rest *= v[k].d;
    }
    // chunks: TI U ~ 64 elements, TO as large as the tile allows, then balanced
    int64_t TI = std::min<int64_t>({Lin, want, kPermTileSide});
    int64_t TO = std::min<int64_t>({Lout, kPermTileElems / (TI * U), kPermTileSide});
    TI = std::min<int64_t>({Lin, kPermTileElems / (TO * U), kPermTileSide});
    const int64_t nci = (Lin + TI - 1) / TI, nco = (Lout + TO - 1) / TO;
    TI = (Lin + nci - 1) / nci;
    TO = (Lout + nco - 1) / nco;
    t.U = (int)U;
    t.TI = (int)TI;
    t.TO = (int)TO;
    t.Lin = (int)Lin;
    t.Lout = (int)Lout;
    t.nci = (int)nci;
    t.nco = (int)nco;
    t.tiles = rest * nci * nco;
    t.fU = make_fastdiv((uint32_t)U);
    t.fci = make_fastdiv((uint32_t)nci);
    t.fco = make_fastdiv((uint32_t)nco);
    t.frun[0] = make_fastdiv((uint32_t)(TI * U));
    t.frun[1] = make_fastdiv((uint32_t)((Lin - (nci - 1) * TI) * U));
    t.fruno[0] = make_fastdiv((uint32_t)(TO * U));
    t.fruno[1] = make_fastdiv((uint32_t)((Lout - (nco - 1) * TO) * U));
    return true;
}

}  // namespace ctmk
