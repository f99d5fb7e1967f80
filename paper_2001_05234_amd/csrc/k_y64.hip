// k_y64.hip -- launcher of the FP64 y transforms.
#include "xform_kernels.h"

namespace cans {

int launch_y_f64(const Problem &pb, bool fwd, const double *in, double *out, hipStream_t s)
{
    const XGeom &g = pb.ay.gy64[fwd ? 1 : 0];
    const int ntx = (pb.nx + g.L - 1) / g.L;
    const dim3 grid((unsigned)(ntx * pb.nz));
    const size_t sh = tile_lds(AX_Y, g, sizeof(double));
    CANS_KIND_SWITCH(pb.ay.kind,
        if (fwd) hipLaunchKernelGGL((k_xform_y<KD, true, double, double>), grid, dim3(kThreads), sh, s,
                                    in, out, pb.nx, pb.ny, ntx, g, pb.ay.d_tw64, nullptr);
        else hipLaunchKernelGGL((k_xform_y<KD, false, double, double>), grid, dim3(kThreads), sh, s,
                                in, out, pb.nx, pb.ny, ntx, g, pb.ay.d_tw64, nullptr));
    return check_launch();
}

int launch_y_f64_grp(const GroupLaunch &gl, bool fwd, hipStream_t s)
{
    const YJob *j = static_cast<const YJob *>(gl.jobs);
    CANS_KIND_SWITCH(gl.key,
        if (fwd) hipLaunchKernelGGL((k_xform_y_grp<KD, true, double, double>), dim3(gl.blocks), dim3(kThreads),
                                    gl.lds, s, j, gl.start, gl.np);
        else hipLaunchKernelGGL((k_xform_y_grp<KD, false, double, double>), dim3(gl.blocks), dim3(kThreads),
                                gl.lds, s, j, gl.start, gl.np));
    return check_launch();
}

}  // namespace cans
