/* Prints the size and field offsets of the ABI's structs, for the CPU test
 * that compares them with the Python binding's ctypes mirrors. */
#include <stddef.h>
#include <stdio.h>

#include "rendermap.h"

#define F(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f))

int main(void) {
    printf("rm_camera %zu\n", sizeof(rm_camera));
    F(rm_camera, fx); F(rm_camera, width); F(rm_camera, z_near); F(rm_camera, z_far);
    printf("rm_mesh %zu\n", sizeof(rm_mesh));
    F(rm_mesh, xyz); F(rm_mesh, n_vertices); F(rm_mesh, tri); F(rm_mesh, cls); F(rm_mesh, n_tris);
    F(rm_mesh, clusters); F(rm_mesh, color);
    printf("rm_scan %zu\n", sizeof(rm_scan));
    F(rm_scan, depth); F(rm_scan, cls); F(rm_scan, mask); F(rm_scan, cam); F(rm_scan, color);
    printf("rm_cost_params %zu\n", sizeof(rm_cost_params));
    F(rm_cost_params, eps); F(rm_cost_params, flags); F(rm_cost_params, color_tol);
    return 0;
}
