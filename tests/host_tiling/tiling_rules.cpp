// Prints the inner solver's tiling rules for the (nx, degree, precision,
// columns, compute units) cases read from stdin, one per line:
//   band_halo band_ntx(nx, degree) band_cols(nx, 1) pcg_band_rows busiest-block tiles
#include <cstdio>
#include "../../paper_1205_1864_amd/csrc/sg_internal.h"

int main() {
  int nx, degree, prec, ncols, ncu;
  while (std::scanf("%d %d %d %d %d", &nx, &degree, &prec, &ncols, &ncu) == 5) {
    const int rows = sgk::pcg_band_rows(nx, degree, prec, ncols, ncu);
    const long ntiles = (long)ncols * sgk::band_ntx(nx, degree) * ((nx + rows - 1) / rows);
    std::printf("%d %d %d %d %ld\n", sgk::band_halo(degree), sgk::band_ntx(nx, degree), sgk::band_cols(nx, 1), rows,
                sgk::pcg_busiest_block(ntiles, ncu));
  }
  return 0;
}
