/* A plain C99 consumer of the library: the header compiles as C with every
 * warning turned into an error, the shared library links, and host-side
 * argument validation answers without touching a GPU. */
#include <stdio.h>
#include <string.h>

#include "txs.h"

int main(void) {
  if (txs_abi_version() != TXS_ABI_VERSION || TXS_ABI_VERSION != 2) return 1;
  /* zero bins are refused on the host, before any launch */
  txs_status st = txs_resample(4, 0, NULL, NULL, TXS_PDF_SIGMA, 8, NULL, NULL, NULL);
  if (st != TXS_EINVAL) return 2;
  if (strstr(txs_last_error(), "n_bins") == NULL) return 3;
  /* a negative ray count is refused too */
  st = txs_compact_rows(-1, NULL, 1, NULL, NULL, NULL);
  if (st != TXS_EINVAL) return 4;
  if (txs_scan_workspace_size(1 << 20) == 0) return 5;
  /* brick occupancy sizes; a zero-initialised grid descriptor has none */
  if (txs_grid_coarse_words(128) != 257 || txs_grid_coarse_words(4) != 0) return 6;
  {
    txs_grid g;
    memset(&g, 0, sizeof g);
    if (g.coarse != NULL) return 7;
  }
  printf("ok\n");
  return 0;
}
