/*
 * A plain C consumer of the library's C ABI: no Python, no torch, only
 * include/pyrit.h, libpyrit.so and the HIP runtime for device memory and a
 * stream.  It encodes one GF(2^8) k=10 m=4 stripe (ragged slice size: several
 * workgroups and a partial one), erases two data and two parity blocks and
 * decodes them back bit for bit, checks that a one-item batch (graph replay
 * and direct dispatch) writes the same parity bytes as the plain encode, and
 * checks two error paths.  Prints "ok" and exits 0 when every check holds.
 * Built by the package's build step; run by tests/test_gpu_c_abi.py.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "pyrit.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);   \
      exit(1);                                                          \
    }                                                                   \
  } while (0)

#define HIP(x)                                                                          \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      fprintf(stderr, "HIP error %s (line %d)\n", hipGetErrorString(e_), __LINE__);     \
      exit(1);                                                                          \
    }                                                                                   \
  } while (0)

enum { W = 8, N = 17, K = 10, M = 4 };
static const uint32_t P = 0x139u;

static uint8_t *host_copy(const uint8_t *dev, size_t bytes) {
  uint8_t *h = (uint8_t *)malloc(bytes);
  CHECK(h != NULL);
  HIP(hipMemcpy(h, dev, bytes, hipMemcpyDeviceToHost));
  return h;
}

int main(void) {
  const size_t S = 64 * (3 * 256 + 5); /* 49 472 bytes per slice */
  const size_t B = (size_t)W * S;
  uint16_t G[M * K];
  pyrit_plan *plan = NULL;
  hipStream_t st;
  uint8_t *blk[K + M], *par2[M];
  int i;

  printf("abi_roundtrip: %s, GF(2^%d) k=%d m=%d, S=%zu\n", pyrit_version(), W, K, M, S);
  fflush(stdout);
  CHECK(pyrit_cauchy(W, P, K, M, G) == PYRIT_OK);
  CHECK(pyrit_plan_create(W, N, P, K, M, G, &plan) == PYRIT_OK);
  HIP(hipStreamCreate(&st));
  for (i = 0; i < K + M; ++i) HIP(hipMalloc((void **)&blk[i], B));
  for (i = 0; i < M; ++i) HIP(hipMalloc((void **)&par2[i], B));
  for (i = 0; i < K; ++i) CHECK(pyrit_fill_random(blk[i], B, B, 4242u + (uint64_t)i, st) == PYRIT_OK);

  /* encode, keep every block on the host */
  CHECK(pyrit_encode(plan, (const uint8_t *const *)blk, blk + K, S, st) == PYRIT_OK);
  HIP(hipStreamSynchronize(st));
  uint8_t *keep[K + M];
  for (i = 0; i < K + M; ++i) keep[i] = host_copy(blk[i], B);

  /* erase data blocks 0 and 3 and parity blocks 11 and 13, decode them */
  const int erased[4] = {0, 3, 11, 13};
  for (i = 0; i < 4; ++i) HIP(hipMemsetAsync(blk[erased[i]], 0, B, st));
  CHECK(pyrit_decode(plan, erased, 4, blk, S, st) == PYRIT_OK);
  HIP(hipStreamSynchronize(st));
  for (i = 0; i < 4; ++i) {
    uint8_t *got = host_copy(blk[erased[i]], B);
    CHECK(memcmp(got, keep[erased[i]], B) == 0);
    free(got);
  }

  /* the same encode as a one-item batch: graph replay, then direct dispatch */
  uint8_t *items_blocks[K + M];
  for (i = 0; i < K; ++i) items_blocks[i] = blk[i];
  for (i = 0; i < M; ++i) items_blocks[K + i] = par2[i];
  pyrit_batch_item item;
  memset(&item, 0, sizeof(item));
  item.plan = plan;
  item.n_erased = 0;
  item.erased = NULL;
  item.blocks = items_blocks;
  item.slice_bytes = S;
  item.slice_pitch = 0;
  pyrit_batch *batch = NULL;
  CHECK(pyrit_batch_create(&item, 1, NULL, &batch) == PYRIT_OK);
  int form;
  for (form = 0; form < 2; ++form) {
    for (i = 0; i < M; ++i) HIP(hipMemsetAsync(par2[i], 0xA5, B, st));
    CHECK((form == 0 ? pyrit_batch_launch(batch, st) : pyrit_batch_launch_direct(batch, st)) ==
          PYRIT_OK);
    HIP(hipStreamSynchronize(st));
    for (i = 0; i < M; ++i) {
      uint8_t *got = host_copy(par2[i], B);
      CHECK(memcmp(got, keep[K + i], B) == 0);
      free(got);
    }
  }
  pyrit_batch_destroy(batch);

  /* error paths: a slice size that is not a multiple of 64, too many erasures */
  CHECK(pyrit_encode(plan, (const uint8_t *const *)blk, blk + K, 100, st) == PYRIT_EALIGN);
  const int five[5] = {0, 1, 2, 3, 4};
  CHECK(pyrit_decode(plan, five, 5, blk, S, st) == PYRIT_ETOOMANY);
  CHECK(pyrit_strerror(PYRIT_ETOOMANY) != NULL);

  for (i = 0; i < K + M; ++i) {
    free(keep[i]);
    HIP(hipFree(blk[i]));
  }
  for (i = 0; i < M; ++i) HIP(hipFree(par2[i]));
  HIP(hipStreamDestroy(st));
  pyrit_plan_destroy(plan);
  printf("ok\n");
  return 0;
}
