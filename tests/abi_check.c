/* A plain C99 program against include/imin.h and libimin.so: the header compiles as strict
 * C, the library links, and the argument checks that precede any device call return the
 * documented status codes (no GPU needed). Built and run by tests/test_abi.py. */
#include <stdio.h>
#include <string.h>
#include "imin.h"
int main(void)
{
    int32_t row_ptr[3] = {0, 1, 1};
    int32_t col[1] = {1};
    float prob[1] = {0.5f};
    imin_graph *g = NULL;
    if (imin_graph_create(0, 0, row_ptr, col, prob, &g) != IMIN_EINVAL || g) return 1;
    prob[0] = 1.5f;
    if (imin_graph_create(2, 1, row_ptr, col, prob, &g) != IMIN_EINVAL || g) return 2;
    if (imin_graph_create_model(2, 1, row_ptr, col, prob, 5, &g) != IMIN_EINVAL || g) return 3;
    if (strcmp(imin_strerror(IMIN_EINVAL), "invalid argument") != 0) return 4;
    if (imin_set_launch(NULL, 1, 1) != IMIN_EINVAL) return 5;
    imin_graph_destroy(NULL);
    printf("c abi ok\n");
    return 0;
}
