// Cooperative walk of one wavefront over the tile rectangles of 64
// consecutive records (the footprint walk and the instance emission of the
// sort).
//
// The rectangles are laid end to end (exclusive prefix `aoff` of their
// areas); chunk j0 .. j0+63 of that sequence goes to lanes 0..63.  The owner
// of position p is the record whose run contains it: every record starting
// inside the chunk writes its lane id into a 64-entry table at its start, a
// ballot over the table marks the starts, and a lane takes the nearest start
// at or below its position (or the record carried over from the previous
// chunk).  The owner's record is read from the wavefront's LDS slice.  Each
// position's tile is then tested against the footprint ellipse
// (tile_hit_rcp) by the caller.
#pragma once

#include "projection.h"

namespace sg {

struct RectRec {
  float mx, my, a, b;     // stored float32 mean and conic
  float c;
  uint32_t xy0;           // rect x0 | y0 << 16
  uint32_t wdt;           // rect width in tiles
  uint32_t aoff;          // start of the record's run
  uint32_t tag0, tag1;    // caller data (record id, tile base / tiles_x ...)
  uint32_t pad0, pad1;
  float ia, ic;           // 1/a, 1/c (filled by rect_walk)
  float iw, pad2;         // 1/width (filled by rect_walk)
};

// The rectangle a record's walk covers: its stored tile rectangle (a square
// of radius 3 sqrt(lambda_max) around the mean) cut down to the tiles whose
// boxes of pixel centres meet the bounding box of the footprint ellipse
// d^T A d <= radius_sigmas^2 (1 + 1e-6) -- the only tiles tile_hit_rcp can
// accept.  The half-widths sqrt(t A^-1_xx), sqrt(t A^-1_yy) come from the
// stored float conic (determinant in fp64, then fp32) and are widened by
// 1e-4 relative and 1e-2 px, far above their rounding.  Fills the record's
// geometry and returns the area (0: nothing to walk).
SG_DEV uint32_t walk_rect(const steepgs_splat& sp, const steepgs_opts& opt, RectRec& me) {
  int x0 = (int)(sp.rect_lo & 0xFFFFu), y0 = (int)(sp.rect_lo >> 16);
  int x1 = (int)(sp.rect_hi & 0xFFFFu), y1 = (int)(sp.rect_hi >> 16);
  const double det = (double)sp.conic_a * (double)sp.conic_c - (double)sp.conic_b * (double)sp.conic_b;
  if (det > 0.0) {
    const float t = opt.radius_sigmas * opt.radius_sigmas * (1.f + 1e-6f);
    const float idet = (float)(1.0 / det);
    const float ex = sqrtf(t * sp.conic_c * idet) * (1.f + 1e-4f) + 1e-2f;
    const float ey = sqrtf(t * sp.conic_a * idet) * (1.f + 1e-4f) + 1e-2f;
    const float tw = (float)opt.tile_w, th = (float)opt.tile_h;
    // tile tx is reachable when tx*tw <= mx + ex and tx*tw + tw - 1 >= mx - ex
    const float lx = ceilf((sp.mean_x - ex - (tw - 1.f)) / tw), hx = floorf((sp.mean_x + ex) / tw);
    const float ly = ceilf((sp.mean_y - ey - (th - 1.f)) / th), hy = floorf((sp.mean_y + ey) / th);
    if (lx > (float)x0) x0 = lx > (float)x1 ? x1 + 1 : (int)lx;
    if (hx < (float)x1) x1 = hx < (float)x0 ? x0 - 1 : (int)hx;
    if (ly > (float)y0) y0 = ly > (float)y1 ? y1 + 1 : (int)ly;
    if (hy < (float)y1) y1 = hy < (float)y0 ? y0 - 1 : (int)hy;
  }
  me.mx = sp.mean_x;
  me.my = sp.mean_y;
  me.a = sp.conic_a;
  me.b = sp.conic_b;
  me.c = sp.conic_c;
  if (x1 < x0 || y1 < y0) {
    me.wdt = 1;
    me.xy0 = 0;
    return 0u;
  }
  me.wdt = (uint32_t)(x1 - x0 + 1);
  me.xy0 = (uint32_t)x0 | ((uint32_t)y0 << 16);
  return me.wdt * (uint32_t)(y1 - y0 + 1);
}

// LDS per wavefront: the 64 records field by field (one array per field, so
// that lanes reading different records hit different banks; a 64-byte record
// per lane put records two apart on the same banks) and the start table.
struct RectWalkLds {
  float mx[64], my[64], a[64], b[64], c[64], ia[64], ic[64], iw[64];
  uint32_t xy0[64], wdt[64], aoff[64], tag0[64], tag1[64], pad0[64];
  int at[64];
  SG_DEV void put(int k, const RectRec& r) {
    mx[k] = r.mx; my[k] = r.my; a[k] = r.a; b[k] = r.b; c[k] = r.c; ia[k] = r.ia; ic[k] = r.ic; iw[k] = r.iw;
    xy0[k] = r.xy0; wdt[k] = r.wdt; aoff[k] = r.aoff; tag0[k] = r.tag0; tag1[k] = r.tag1; pad0[k] = r.pad0;
  }
  SG_DEV RectRec get(int k) const {
    RectRec r;
    r.mx = mx[k]; r.my = my[k]; r.a = a[k]; r.b = b[k]; r.c = c[k]; r.ia = ia[k]; r.ic = ic[k]; r.iw = iw[k];
    r.xy0 = xy0[k]; r.wdt = wdt[k]; r.aoff = aoff[k]; r.tag0 = tag0[k]; r.tag1 = tag1[k]; r.pad0 = pad0[k];
    r.pad1 = 0u; r.pad2 = 0.f;
    return r;
  }
};

// Sets up a wavefront's walk: the records go to the wavefront's LDS slice,
// each lane gets the start of its own run (aoff).  Returns the total area
// (uniform over the wavefront).
SG_DEV uint32_t rect_walk_begin(RectWalkLds& L, int lane, uint32_t area, const RectRec& mine, uint32_t& aoff) {
  uint32_t incl = area;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const uint32_t atotal = __shfl(incl, 63, 64);
  aoff = incl - area;
  RectRec me = mine;
  me.aoff = aoff;
  me.ia = 1.f / me.a;
  me.ic = 1.f / me.c;
  me.iw = 1.f / (float)me.wdt;
  L.put(lane, me);
  return atotal;
}

// Position j0 + lane of the walk (area, aoff: the lane's own record): returns
// the owner lane, i.e. the lane whose record's run holds the position, and
// its tile (tx, ty).  `carry` is the owner of the previous chunk's last
// position (0 before the first chunk).  Every lane of the wavefront takes part.
SG_DEV int rect_walk_locate(RectWalkLds& L, int lane, uint32_t area, uint32_t aoff, uint32_t j0, int& carry, int& tx,
                            int& ty) {
  // starts of the records inside this chunk
  L.at[lane] = -1;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (area > 0 && aoff >= j0 && aoff - j0 < 64u) L.at[aoff - j0] = lane;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint64_t starts = ballot(L.at[lane] >= 0);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const uint64_t below = starts & upto;
  const int owner = below ? L.at[63 - __builtin_clzll(below)] : carry;
  carry = __builtin_amdgcn_readlane(owner, 63);
  const uint32_t q = j0 + (uint32_t)lane - L.aoff[owner];
  const uint32_t wdt = L.wdt[owner], xy0 = L.xy0[owner];
  const float iw = L.iw[owner];
  // q / width without an integer division: the float quotient is off by at
  // most one for q < 2^24, fixed up exactly below (larger q: integer path)
  int row, col;
  if (q < (1u << 24)) {
    row = (int)((float)q * iw);
    col = (int)q - row * (int)wdt;
    if (col < 0) {
      --row;
      col += (int)wdt;
    } else if (col >= (int)wdt) {
      ++row;
      col -= (int)wdt;
    }
  } else {
    row = (int)(q / wdt);
    col = (int)(q % wdt);
  }
  tx = (int)(xy0 & 0xFFFFu) + col;
  ty = (int)(xy0 >> 16) + row;
  return owner;
}

}  // namespace sg
