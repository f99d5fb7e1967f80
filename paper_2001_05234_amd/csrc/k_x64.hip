// k_x64.hip -- launcher of the FP64 x transforms.
#include "xform_kernels.h"

namespace cans {

int launch_x_f64(const Problem &pb, bool fwd, const double *in, double *out, hipStream_t s)
{
    const XGeom &g = pb.ax.gx64[fwd ? 1 : 0];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)((nlines + g.L - 1) / g.L));
    const size_t sh = tile_lds(AX_X, g, sizeof(double));
    CANS_KIND_SWITCH(pb.ax.kind,
        if (fwd) hipLaunchKernelGGL((k_xform_x<KD, true, double, double, double, 0>), grid, dim3(kThreads), sh, s,
                                    in, out, nlines, g, pb.ax.d_tw64, nullptr, nullptr, nullptr, pb.ny, nullptr);
        else hipLaunchKernelGGL((k_xform_x<KD, false, double, double, double, 0>), grid, dim3(kThreads), sh, s,
                                in, out, nlines, g, pb.ax.d_tw64, nullptr, nullptr, nullptr, pb.ny, nullptr));
    return check_launch();
}


int launch_x_f64_grp(const GroupLaunch &gl, bool fwd, hipStream_t s)
{
    const XJob *j = static_cast<const XJob *>(gl.jobs);
    CANS_KIND_SWITCH(gl.key,
        if (fwd) hipLaunchKernelGGL((k_xform_x_grp<KD, true, double, double, double, 0>), dim3(gl.blocks),
                                    dim3(kThreads), gl.lds, s, j, gl.start, gl.np);
        else hipLaunchKernelGGL((k_xform_x_grp<KD, false, double, double, double, 0>), dim3(gl.blocks),
                                dim3(kThreads), gl.lds, s, j, gl.start, gl.np));
    return check_launch();
}

}  // namespace cans
