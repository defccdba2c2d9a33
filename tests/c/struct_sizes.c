/* Prints the size of every struct of the C ABI (include/npt.h), one
 * "name size" line each, so that tests/test_abi_c.py can check the Python
 * binding's ctypes mirrors against the C compiler's layout. */
#include <stdio.h>

#include "npt.h"

#define SIZE(T) printf("%s %zu\n", #T, sizeof(T))

int main(void) {
    SIZE(npt_material);
    SIZE(npt_instance);
    SIZE(npt_camera);
    SIZE(npt_bvh_params);
    SIZE(npt_nif_desc);
    SIZE(npt_train_params);
    SIZE(npt_train_stats);
    SIZE(npt_render_options);
    SIZE(npt_stats);
    return 0;
}
