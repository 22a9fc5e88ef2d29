/* A plain C client of the library: builds a host-only grid from a mask
 * through the C ABI and checks what it reports, with no Python in the way.
 * Exit status 0 on success; prints the first failing check otherwise. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gpe.h"

#define CHECK(cond, what)                                         \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "check failed: %s (%s)\n", what, gpe_last_error()); \
      return 1;                                                   \
    }                                                             \
  } while (0)

int main(void) {
  const int64_t n0 = 6, n1 = 5, n2 = 7;
  gpe_geometry geom = {{n0, n1, n2}, {0.5, 0.5, 0.5}, {-1.5, -1.25, -1.75}};
  uint8_t* mask = (uint8_t*)calloc((size_t)(n0 * n1 * n2), 1);
  int64_t expect = 0;
  for (int64_t i = 0; i < n0; ++i)
    for (int64_t j = 0; j < n1; ++j)
      for (int64_t k = 0; k < n2; ++k)
        if ((i * 7 + j * 3 + k * 5) % 4 != 0) {   /* a ragged pattern */
          mask[(i * n1 + j) * n2 + k] = 1;
          ++expect;
        }
  gpe_grid g = NULL;
  CHECK(gpe_abi_version() == GPE_ABI_VERSION, "abi version");
  CHECK(gpe_grid_create(&geom, mask, -1, &g) == GPE_OK, "create host-only grid");
  int64_t na = 0, nr = 0, ns = 0;
  CHECK(gpe_grid_info(g, &na, &nr, &ns) == GPE_OK, "info");
  CHECK(na == expect, "active count");
  /* the segment table tiles the active sites exactly once */
  int32_t* segs = (int32_t*)malloc(sizeof(int32_t) * 8 * (size_t)ns);
  CHECK(gpe_grid_segments(g, segs) == GPE_OK, "segments");
  int64_t covered = 0;
  for (int64_t q = 0; q < ns; ++q) {
    CHECK(segs[8 * q] == covered, "segments are contiguous");
    covered += segs[8 * q + 1];
  }
  CHECK(covered == na, "segments cover the active set");
  /* work sizes: RK4 stores three states, RKHE3 two, RKCK five */
  size_t b3 = 0, b2 = 0, b5 = 0;
  CHECK(gpe_work_bytes(g, GPE_C128, GPE_MODE_RT, 10, 0, &b3) == GPE_OK, "work RK4");
  CHECK(gpe_work_bytes(g, GPE_C128, GPE_MODE_RT_RKHE3, 10, 0, &b2) == GPE_OK, "work RKHE3");
  CHECK(gpe_work_bytes(g, GPE_C128, GPE_MODE_RT_RKCK, 10, 0, &b5) == GPE_OK, "work RKCK");
  CHECK(b2 < b3 && b3 < b5, "work sizes ordered");
  /* stencil selection is recorded, 27 points need equal spacings (they are) */
  int32_t pts = 0;
  CHECK(gpe_grid_set_stencil(g, 27) == GPE_OK, "set 27-point stencil");
  CHECK(gpe_grid_get_stencil(g, &pts) == GPE_OK && pts == 27, "get stencil");
  CHECK(gpe_grid_set_stencil(g, 9) == GPE_ERR_ARG, "reject a 9-point stencil");
  int64_t nh = 0;
  CHECK(gpe_grid_stencil_segments(g, 19, &nh, NULL) == GPE_OK && nh >= ns, "19-point table");
  /* compute calls on a host-only grid are refused before any launch */
  gpe_params prm;
  memset(&prm, 0, sizeof prm);
  prm.g = 1.0;
  prm.dt = 1e-3;
  gpe_potential pot;
  memset(&pot, 0, sizeof pot);
  pot.field = mask;
  CHECK(gpe_imag_time(g, GPE_C128, mask, &pot, &prm, 1, mask, 1 << 20, NULL, NULL, NULL) == GPE_ERR_STATE,
        "host-only grid refuses compute");
  CHECK(gpe_grid_destroy(g) == GPE_OK, "destroy");
  free(segs);
  free(mask);
  printf("ok %lld active sites, %lld runs, %lld segments\n", (long long)na, (long long)nr, (long long)ns);
  return 0;
}
