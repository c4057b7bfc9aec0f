/* Prints sizeof and field offsets of the C-ABI structs, as the C compiler
 * lays them out from include/ccl.h. */
#include <stddef.h>
#include <stdio.h>

#include "../../include/ccl.h"

#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
#define S(T) printf(#T " %zu\n", sizeof(T))

int main(void) {
  S(ccl_feature_t); F(ccl_feature_t, S); F(ccl_feature_t, Sy);
  S(ccl_outputs_t); F(ccl_outputs_t, cap); F(ccl_outputs_t, counts);
  S(ccl_image_t); F(ccl_image_t, pitch); F(ccl_image_t, out);
  S(ccl_server_config_t); F(ccl_server_config_t, variant); F(ccl_server_config_t, cap_divisor);
  S(ccl_done_t); F(ccl_done_t, status); F(ccl_done_t, launches); F(ccl_done_t, n_labels); F(ccl_done_t, euler);
  F(ccl_done_t, out);
  S(ccl_server_stats_t); F(ccl_server_stats_t, ready); F(ccl_server_stats_t, relaunched);
  return 0;
}
