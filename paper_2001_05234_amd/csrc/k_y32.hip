// k_y32.hip -- launcher of the FP32 y transforms of the refinement path.
#include "xform_kernels.h"

namespace cans {

int launch_y_32(const Problem &pb, bool fwd, float *data, const int *done, hipStream_t s)
{
    const XGeom &g = pb.ay.gy32[fwd ? 1 : 0];
    const int ntx = (pb.nx + g.L - 1) / g.L;
    const dim3 grid((unsigned)(ntx * pb.nz));
    const size_t sh = tile_lds(AX_Y, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ay.kind,
        if (fwd) hipLaunchKernelGGL((k_xform_y<KD, true, float, float>), grid, dim3(kThreads), sh, s,
                                    data, data, pb.nx, pb.ny, ntx, g, pb.ay.d_tw32, done);
        else hipLaunchKernelGGL((k_xform_y<KD, false, float, float>), grid, dim3(kThreads), sh, s,
                                data, data, pb.nx, pb.ny, ntx, g, pb.ay.d_tw32, done));
    return check_launch();
}


int launch_y_32_grp(const GroupLaunch &gl, bool fwd, hipStream_t s)
{
    const YJob *j = static_cast<const YJob *>(gl.jobs);
    CANS_KIND_SWITCH(gl.key,
        if (fwd) hipLaunchKernelGGL((k_xform_y_grp<KD, true, float, float>), dim3(gl.blocks), dim3(kThreads),
                                    gl.lds, s, j, gl.start, gl.np);
        else hipLaunchKernelGGL((k_xform_y_grp<KD, false, float, float>), dim3(gl.blocks), dim3(kThreads),
                                gl.lds, s, j, gl.start, gl.np));
    return check_launch();
}

}  // namespace cans
