/* Calls the library's host-only entry points from plain C (C11): the header
 * must compile as C and the exported symbols must link.  Prints "ok". */
#include <stdio.h>
#include <string.h>

#include "lb.h"

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void)
{
    CHECK(lb_abi_version() == LB_ABI_VERSION);
    CHECK(strcmp(lb_status_string(LB_OK), "ok") == 0);
    const int32_t *fake = (const int32_t *)0x10000; /* never dereferenced */
    lb_csr_t A = {1000, 1000, 5000, fake, fake, fake, LB_F32};
    lb_schedule_t in = {LB_AUTO, 0, 0, 0, 0, 0}, out;
    CHECK(lb_resolve_schedule(&A, 1, &in, &out) == LB_OK);
    /* a small matrix (6000 merge items): the shortest default units, 128 x 4 */
    CHECK(out.kind == LB_MERGE_PATH && out.block_size == 128 && out.items_per_thread == 4);
    size_t ws = 0;
    CHECK(lb_workspace_size(&A, &out, 1, &ws) == LB_OK && ws > 0);
    lb_schedule_t bad = {LB_GROUP_MAPPED, 3, 0, 0, 0, 0};
    CHECK(lb_resolve_schedule(&A, 1, &bad, &out) == LB_ERR_INVALID_ARG);
    CHECK(lb_spmv(&A, fake, LB_F32, (float *)fake, &in, (void *)fake, 4, NULL) == LB_ERR_WORKSPACE_TOO_SMALL);
    lb_csr_t big = {1 << 30, 10, 1 << 30, fake, fake, fake, LB_F32};
    CHECK(lb_spmv(&big, fake, LB_F32, (float *)fake, &in, (void *)fake, ws, NULL) == LB_ERR_OVERFLOW);
    lb_csr_t empty = {0, 5, 0, NULL, NULL, NULL, LB_F32};
    CHECK(lb_spmv(&empty, NULL, LB_F32, NULL, &in, NULL, 0, NULL) == LB_OK);
    CHECK(lb_merge_path_partition(NULL, 1, 1, 1, 1, (int32_t *)fake, (int32_t *)fake, NULL) == LB_ERR_INVALID_ARG);
    lb_csr_t tall = {5000000, 5000000, 10000000, fake, fake, fake, LB_F32};
    lb_schedule_t banded = {LB_MERGE_PATH, 0, 0, 0, 0, 0, 2, 0};
    CHECK(lb_spmv_noalloc(&tall, fake, LB_F32, (float *)fake, &banded, NULL) == LB_ERR_SCRATCH_LIMIT);
    puts("ok");
    return 0;
}
