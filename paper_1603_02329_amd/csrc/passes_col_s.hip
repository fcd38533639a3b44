// Column-pass instances for the short axes (16 to 128 points) and the host
// side of the column passes: launch variants, blocks per instance, dispatch.
#include "passes_col.h"

namespace pat {

hipError_t launch_col_long(const ColSpec& spec, ColVariant v, int na, const Launch& L);
hipError_t upload_twiddles_cols_long(const Tw* host);

static int default_tile(int na) {
  switch (na) {
    case 16: return ColGeo<16>::TILE;
    case 32: return ColGeo<32>::TILE;
    case 64: return ColGeo<64>::TILE;
    case 128: return ColGeo<128>::TILE;
    case 256: return ColGeo<256>::TILE;
    case 512: return ColGeo<512>::TILE;
    case 1024: return ColGeo<1024>::TILE;
  }
  return 0;
}

int col_axis_len(const ColSpec& spec, int ndim, int ny, int nz) {
  return (ndim == 2 || spec.mode >= 3) ? ny : nz;
}

// The default (as many columns as fit 1024 threads, at most 16; mode 1 one
// field per block) first.  Multiplier passes with columns of 128 to 512
// points and one or two fields per launch also have 8 and 4 columns per
// block, and mode-1 passes over two fields can take both in one block.
int col_variants(const ColSpec& spec, int ndim, int ny, int nz, ColVariant* out) {
  const int na = col_axis_len(spec, ndim, ny, nz);
  const int d = default_tile(na);
  if (!d) return 0;
  int n = 0;
  out[n++] = ColVariant{d, 1};
  if (spec.mode == 3 || spec.mode == 4 || !col_tunable(na)) return n;
  const bool two = spec.nfield == 2;
  if (spec.mode != 1 && !two) return n;
  const int tiles[3] = {d, 8, 4};
  for (int i = 0; i < 3; ++i) {
    if (i > 0 && tiles[i] == d) continue;
    if (i > 0) out[n++] = ColVariant{tiles[i], 1};
    if (spec.mode == 1 && two) out[n++] = ColVariant{tiles[i], 2};
  }
  return n;
}

ColVariant col_variant_of(const ColSpec& spec, int ndim, int ny, int nz) {
  ColVariant v[kMaxColVar];
  const int n = col_variants(spec, ndim, ny, nz, v);
  for (int i = 0; i < n; ++i)
    if (v[i].tile == spec.tile && v[i].fpb == spec.fpb) return v[i];
  return n ? v[0] : ColVariant{0, 1};
}

// blocks of one column-pass launch for one instance (along grid.x): y-axis
// passes use nz groups of tiles, z-axis passes ny groups
int col_blocks(const ColSpec& spec, int ndim, int nx, int ny, int nz) {
  const int M = nx / 2;
  const int w = col_variant_of(spec, ndim, ny, nz).tile;
  if (!w) return 0;
  const bool along_y = (ndim == 2 || spec.mode >= 3);
  const int other = (ndim == 2) ? 1 : (along_y ? nz : ny);
  return other * ((M + w - 1) / w);
}

hipError_t launch_col(const ColSpec& spec, int ndim, int nx, int ny, int nz, const Launch& L) {
  (void)nx;
  const int na = col_axis_len(spec, ndim, ny, nz);
  const ColVariant v = col_variant_of(spec, ndim, ny, nz);
  switch (na) {
    case 16: return launch_col_na<16>(spec, v, L);
    case 32: return launch_col_na<32>(spec, v, L);
    case 64: return launch_col_na<64>(spec, v, L);
    case 128: return launch_col_na<128>(spec, v, L);
  }
  return launch_col_long(spec, v, na, L);
}

hipError_t upload_twiddles_cols(const Tw* host) {
  const hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof(Tw) * TWN, 0, hipMemcpyHostToDevice);
  return e != hipSuccess ? e : upload_twiddles_cols_long(host);
}

}  // namespace pat
