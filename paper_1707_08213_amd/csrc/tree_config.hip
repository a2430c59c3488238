// Launch shape of the fused tree forward kernel: lanes per column stream,
// slab length, resident-wave cap and tile order, chosen from the plan, the
// SWDFT_TREE_* environment overrides and the device.
#include <algorithm>
#include <cstdlib>

#include "plan.h"

namespace swdft {
namespace host {

namespace {

// Attribute of the current device, cached per device; 0 when there is none.
int device_attr(hipDeviceAttribute_t attr, int (&cache)[64]) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, attr, dev) != hipSuccess || v <= 0) v = -1;
    cache[dev] = v;
  }
  return cache[dev] > 0 ? cache[dev] : 0;
}

}  // namespace

int env_int(const char* name, int fallback) {
  const char* e = std::getenv(name);
  return e && *e ? std::atoi(e) : fallback;
}

int lds_per_cu() {
  static int cache[64] = {};
  return device_attr(hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, cache);
}

int cu_count() {
  static int cache[64] = {};
  return device_attr(hipDeviceAttributeMultiprocessorCount, cache);
}

namespace {

// A small image: even one-chunk slabs give fewer tiles than CUs with the
// default split, so the time is that of one wave's walk down its slab.
bool small_image(const swdft2d_plan_s* p) {
  const int kg = swdft::tree_fwd_default_kg(p->n0, p->n1);
  const int64_t ncu = cu_count() > 0 ? cu_count() : 256;
  const int64_t strips = ceil_div(p->P1, swdft::tree_fwd_columns_per_wave(p->n0, p->n1, kg));
  const int64_t slabs = ceil_div(p->P0, swdft::tree_fwd_rows_per_chunk(p->n0, p->n1, kg, 1));
  return strips * slabs * p->batch < ncu;
}

// Launch of a small image. Its time is that of the longest walk of a wave
// down its slab, and the walk costs mostly per wave: set-up, the row phase of
// a chunk, and steps that do not pipeline with one wave per SIMD. The n0 - 1
// priming rows at a slab top cost little, since they compute only the column
// levels the slab's windows use. Two rules (100 x 100, measured on gfx950):
//  - n0 <= 16: whole streams, one wave per strip and one-chunk slabs (each
//    wave one chunk of rows: mostly priming, then its few windows), as long
//    as the waves fit eight to a CU (16 x 16 7.0 -> 6.3 us, 8 x 8 4.4 ->
//    4.1 us);
//  - otherwise: streams split over two lanes and two waves where built, and
//    the shortest slabs that keep to one workgroup per CU (32 x 32 14.5 ->
//    12.0 us).
struct SmallCfg {
  bool one_chunk = false;  // first rule
  int kg = 1, wv = 1;
};

SmallCfg small_image_cfg(const swdft2d_plan_s* p) {
  SmallCfg c;
  const int64_t ncu = cu_count() > 0 ? cu_count() : 256;
  if (p->n0 <= 16) {
    const int cr = swdft::tree_fwd_rows_per_chunk(p->n0, p->n1, 1, 1);
    const int64_t S = std::max(1, cr - (p->n0 - 1));
    const int64_t strips = ceil_div(p->P1, swdft::tree_fwd_columns_per_wave(p->n0, p->n1, 1));
    if (strips * ceil_div(p->P0, S) * p->batch <= 8 * ncu) {
      c.one_chunk = true;
      return c;
    }
  }
  c.kg = swdft::tree_fwd_default_kg(p->n0, p->n1);
  if (p->n0 < 64 && swdft::tree_fwd_kg_supported(p->n0, p->n1, 2)) c.kg = 2;
  c.wv = swdft::tree_fwd_wv_supported(p->n0, c.kg, 2) ? 2 : 1;
  return c;
}

int32_t tree_kg(const swdft2d_plan_s* p) {
  if (mixed_window(p)) return 1;  // the mixed-radix kernels keep streams whole
  int kg = p->tree_kg > 0 ? p->tree_kg : env_int("SWDFT_TREE_KG", 0);
  if (kg <= 0 || !swdft::tree_fwd_kg_supported(p->n0, p->n1, kg))
    kg = small_image(p) ? small_image_cfg(p).kg : swdft::tree_fwd_default_kg(p->n0, p->n1);
  return kg;
}

// Slab count that fills the rounds of `slots` resident waves to at least 90%
// with `columns` strips (at most 8 slabs), or 0 if none does.
int64_t filling_slabs(int64_t columns, int64_t slots) {
  for (int64_t s = 1; s <= 8; ++s) {
    const int64_t tiles = columns * s;
    if (tiles * 10 >= ceil_div(tiles, slots) * slots * 9) return s;
  }
  return 0;
}

// Resident-wave cap per CU (0 = none) and the slab count that goes with it.
// With one wave per CU, unsplit n0 = 16 streams and a wave per column of its
// strip, the resident waves write one narrow band of output rows that moves
// down the image, which the HBM3E stacks absorb at close to the copy rate;
// with many resident waves the store streams of many tiles interleave and
// the write rate drops by 10-15% (measured on gfx950). The cap is only worth
// it when the rounds of resident waves are nearly full.
struct TreeCap {
  int wpc = 0;
  int64_t slabs = 0;  // 0: slab length from the uncapped rule
};

// Shapes whose default is one workgroup per CU (measured on gfx950): unsplit
// n0 = 16 and n0 = 32 streams (n1 >= 16), split streams of n1 = 8 windows
// (n0 >= 16) with two waves per strip, and n0 = 64 with n1 <= 8. The other
// radix-2 shapes default to two per CU.
bool capped_by_default(int n0, int n1, int kg) {
  return (n0 == 16 && kg == 1) || (n0 >= 16 && n1 == 8 && kg == 2) || (n0 == 32 && kg == 1) ||
         (n0 == 64 && n1 <= 8);
}

// Two waves per strip: capped n1 = 8 split streams, 32 x 32 unsplit (1024^2:
// 1550 -> 1475 us) and n0 = 64 with n1 <= 8 (64 x 8: 774 -> 681 us).
bool two_waves_by_default(int n0, int n1, int kg) {
  return (n0 >= 16 && n1 == 8 && kg == 2) || (n0 == 32 && n1 == 32 && kg == 1) ||
         (n0 == 64 && n1 <= 8);
}

TreeCap tree_cap(const swdft2d_plan_s* p, int kg) {
  const int64_t columns =
      ceil_div(p->P1, swdft::tree_fwd_columns_per_wave(p->n0, p->n1, kg)) * p->batch;
  const int64_t ncu = cu_count() > 0 ? cu_count() : 256;
  TreeCap c;
  c.wpc = p->tree_wpc >= 0 ? p->tree_wpc : env_int("SWDFT_TREE_WPC", -1);
  if (c.wpc < 0) {
    c.wpc = 0;
    // small images: no cap, their many short tiles run at once
    if (small_image(p) && !mixed_window(p)) return c;
    // one resident workgroup per CU for the shapes above; two for the others
    // (1024 x 1024, alternating A/B: 8 x 8 102 -> 85-92 us, 8 x 16 198 -> 193 us), and for
    // mixed-radix windows of 12 x 12 and up (12 x 12 259 -> 246 us, 24 x 24
    // 1026 -> 914 us); none where the rounds would not fill
    int wpc = 0;
    if (mixed_window(p)) {
      wpc = p->n0 * p->n1 >= 144 ? 2 : 0;
      // about one tile per CU when the strips, in one or two slabs, fill one
      // round of CUs (1024 x 1024: 12 x 16 319 -> 278 us, 24 x 8 322 -> 274 us)
      for (int64_t s = 1; wpc == 2 && s <= 2; ++s)
        if (columns * s <= ncu && columns * s * 10 >= ncu * 9) return TreeCap{2, s};
    } else {
      wpc = capped_by_default(p->n0, p->n1, kg) ? 1 : 2;
      // 16 x 16 windows whose whole columns need more than one round of
      // resident waves: slabs of about 48 rows instead, in dispatch order, so
      // that each round of waves writes one band of rows and the last round
      // is short (the priming rows of a slab cost little); measured against
      // whole columns: 16 x 256^2 349 -> 321 us, 2 x 1024^2 706 -> 656 us,
      // 2048^2 1516 -> 1373 us, 4 x 512^2 348 -> 326 us (32 or 64 rows were
      // slower; 16 x 32 windows keep their rule)
      if (p->n0 == 16 && p->n1 == 16 && kg == 1 && columns > ncu)
        return TreeCap{1, std::max<int64_t>(1, ceil_div(p->P0, 48))};
      // likewise 64-row slabs for the two-wave n1 = 8 shapes (split streams
      // for n0 = 16 and 32, whole ones for n0 = 64): 2048^2 / 16x8 790 ->
      // 692 us, 1024^2 / 64x8 735 -> 652 us
      if (p->n1 == 8 && ((p->n0 >= 16 && p->n0 <= 32 && kg == 2) || p->n0 == 64) &&
          columns > ncu)
        return TreeCap{1, std::max<int64_t>(1, ceil_div(p->P0, 64))};
      // short windows with rows of 8 to 32 values: two per CU in 64-row slabs
      // rather than the fewest slabs that fill the rounds (1024^2: 8 x 8 98
      // -> 86 us, 8 x 16 198 -> 169 us, 4 x 8 61 -> 57 us, 4 x 16 105 -> 94
      // us, 8 x 32 375 -> 360 us; 4 x 32 is 187 -> 194 us and n1 = 4 gains
      // nothing, so both keep the fewest slabs)
      if ((p->n0 == 8 && p->n1 >= 8 && p->n1 <= 32) || (p->n0 == 4 && (p->n1 == 8 || p->n1 == 16)))
        return TreeCap{2, std::max<int64_t>(1, ceil_div(p->P0, 64))};
    }
    if (wpc > 0) {
      const int64_t s = filling_slabs(columns, ncu * wpc);
      if (s > 0) c = TreeCap{wpc, s};
    }
    return c;
  }
  c.wpc = std::min(c.wpc, 8);
  if (c.wpc > 0) c.slabs = std::max<int64_t>(1, filling_slabs(columns, ncu * c.wpc));
  return c;
}

// Waves per workgroup sharing a strip: two for the capped shapes of
// two_waves_by_default (one wave's issue rate would bound the tile:
// 1024x1024 / 16x8 went from 5.5 to 6.7-6.9 TB/s, 2048x512 / 32x8 from 5.4 to
// 5.55); one otherwise (for unsplit n0 = 16 streams a second wave lowered the
// write rate by 11%).
int32_t tree_wv(const swdft2d_plan_s* p, int kg, int wpc) {
  if (mixed_window(p)) return 1;
  int wv = p->tree_wv > 0 ? p->tree_wv : env_int("SWDFT_TREE_WV", 0);
  if (wv <= 0) {
    wv = (wpc == 1 && two_waves_by_default(p->n0, p->n1, kg)) ? 2 : 1;
    if (small_image(p)) wv = small_image_cfg(p).wv;
  }
  if (!swdft::tree_fwd_wv_supported(p->n0, kg, wv)) wv = 1;
  if (!swdft::tree_fwd_wv_supported(p->n0, kg, wv)) wv = 2;  // n0 = 64 unsplit: two waves only
  return wv;
}

// Output rows per wave of the fused tree: P0 / slabs for a capped launch;
// otherwise enough tiles (about 4096) to fill the chip several times over,
// with slabs long enough that the n0-1 priming rows at the top of each stay a
// small fraction of the work.
int32_t tree_slab(const swdft2d_plan_s* p, int kg, int wv, const TreeCap& cap) {
  const int cr = tree_chunk_rows(p, kg, wv);
  const int64_t nstrips = ceil_div(p->P1, swdft::tree_fwd_columns_per_wave(p->n0, p->n1, kg));
  int64_t S = p->tree_slab > 0 ? p->tree_slab : env_int("SWDFT_TREE_SLAB", 0);
  if (small_image(p) && !mixed_window(p)) {
    // Small images (small_image_cfg): one-chunk slabs for whole streams on
    // one wave per strip under the first rule; otherwise the shortest slabs
    // that keep to one workgroup per CU. A slab need not be a whole number
    // of chunks (long chunks skip the steps past its end).
    if (S <= 0) {
      const SmallCfg sc = small_image_cfg(p);
      if (sc.one_chunk && kg == 1 && wv == 1) {
        S = std::max(1, cr - (p->n0 - 1));
      } else {
        const int64_t ncu = cu_count() > 0 ? cu_count() : 256;
        S = p->P0;
        for (int64_t s = 1; s <= p->P0; ++s) {
          if (nstrips * ceil_div(p->P0, s) * p->batch <= ncu) {
            S = s;
            break;
          }
        }
      }
    }
    return (int32_t)std::min<int64_t>(S, p->P0);
  }
  if (S <= 0) {
    if (cap.wpc > 0 && cap.slabs > 0) {
      S = ceil_div(p->P0, cap.slabs);
    } else {
      // about 4096 tiles; about 1024 for the uncapped mixed-radix windows
      // (1024 x 1024 / 9 x 9, alternating A/B: 159-165 -> 138-142 us)
      const int64_t tiles = mixed_window(p) ? 1024 : 4096;
      S = ceil_div(p->P0 * nstrips * p->batch, tiles);
      S = std::max<int64_t>(S, 4 * (int64_t)(p->n0 - 1));
      // Small images: rather one chunk per slab (priming rows and all) than
      // fewer tiles than CUs, whose sequential walks down the slab then set
      // the time (100 x 100 / 16 x 16 has 22 strips: 44 tiles of 79 rows, or
      // 132 of 31 with one-chunk slabs).
      const int64_t ncu = cu_count() > 0 ? cu_count() : 256;
      if (nstrips * p->batch * ceil_div(p->P0, ceil_div(S, cr) * cr) < ncu) S = cr;
    }
  }
  S = std::max<int64_t>(S, cr);
  S = ceil_div(S, cr) * cr;
  S = std::min<int64_t>(S, ceil_div(p->P0, cr) * cr);
  return (int32_t)S;
}

}  // namespace

bool mixed_window(const swdft2d_plan_s* p) { return !is_pow2(p->n0) || !is_pow2(p->n1); }

int tree_chunk_rows(const swdft2d_plan_s* p, int kg, int wv) {
  return mixed_window(p) ? swdft::tree_mixed_rows_per_chunk(p->n0, p->n1)
                         : swdft::tree_fwd_rows_per_chunk(p->n0, p->n1, kg, wv);
}

swdft::TreeGeom tree_geom(const swdft2d_plan_s* p) {
  swdft::TreeGeom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.x_image_stride = p->N0 * p->N1;
  g.y_image_stride = p->P0 * p->P1 * p->n0 * p->n1;
  g.kg = tree_kg(p);
  const TreeCap cap = tree_cap(p, g.kg);
  g.wpc = cap.wpc;
  g.wv = tree_wv(p, g.kg, g.wpc);
  g.S = tree_slab(p, g.kg, g.wv, cap);
  g.nstrips = (int32_t)ceil_div(p->P1, swdft::tree_fwd_columns_per_wave(p->n0, p->n1, g.kg));
  g.nslabs = (int32_t)ceil_div(p->P0, g.S);
  g.batch = (int32_t)p->batch;
  g.scale = norm_scale(p->norm, p->n0, p->n1);
  g.lds_cu = lds_per_cu();
  // With a cap and more tiles than one round of resident waves, tiles run in
  // dispatch order so that each round covers one contiguous range of strips;
  // otherwise each XCD takes a contiguous range (neighbouring strips share
  // input columns in that XCD's L2).
  const int64_t tiles = (int64_t)g.nstrips * g.nslabs * g.batch;
  const int64_t resident = (int64_t)swdft::tree_fwd_resident_waves(g.wpc, cu_count());
  g.order = (g.wpc > 0 && resident > 0 && tiles > resident) ? 1 : 0;
  if (g.lds_cu <= 0) g.wpc = 0;
  return g;
}

const swdft::TreeGeom& tree_geom_cached(swdft2d_plan_s* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  const int32_t key[10] = {dev,
                           p->tree_kg,
                           p->tree_wpc,
                           p->tree_wv,
                           p->tree_slab,
                           (int32_t)p->norm,
                           env_int("SWDFT_TREE_KG", 0),
                           env_int("SWDFT_TREE_WPC", -1),
                           env_int("SWDFT_TREE_WV", 0),
                           env_int("SWDFT_TREE_SLAB", 0)};
  if (!p->tree_geom_valid || !std::equal(key, key + 10, p->tree_geom_key)) {
    p->tree_geom_last = tree_geom(p);
    std::copy(key, key + 10, p->tree_geom_key);
    p->tree_geom_valid = true;
  }
  return p->tree_geom_last;
}

}  // namespace host
}  // namespace swdft
