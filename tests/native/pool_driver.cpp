// Replays an allocation trace against ccl::Pool (the serving loop's
// sub-allocator) on the host.  stdin: "size BYTES", then lines "a N" (alloc)
// or "r OFF N" (release); stdout: one line per alloc with the offset or -1,
// and after every operation the pool's used bytes and free-block count.
#include <stdio.h>

#include "../../paper_2006_09299_amd/csrc/ccl_pool.h"

int main() {
  unsigned long long size = 0;
  if (scanf(" size %llu", &size) != 1) return 2;
  ccl::Pool p(size);
  char op;
  while (scanf(" %c", &op) == 1) {
    unsigned long long a = 0, b = 0;
    if (op == 'a') {
      if (scanf("%llu", &a) != 1) return 2;
      size_t off = p.alloc(a);
      printf("%lld", off == ccl::Pool::NONE ? -1LL : (long long)off);
    } else if (op == 'r') {
      if (scanf("%llu %llu", &a, &b) != 2) return 2;
      p.release(a, b);
      printf("r");
    } else {
      return 2;
    }
    printf(" %zu %zu %zu\n", p.used(), p.free_blocks(), p.largest_free());
  }
  return 0;
}
