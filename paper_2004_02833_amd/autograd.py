"""torch.autograd.Function around the C ABI: forward runs the P_N steps,
backward runs the library's transposed steps (pm_grad_dev).

Torch supplies tensors and the stream only; all arithmetic runs in libpm.
The library holds one global context, so a forward must be followed by its
backward before the next forward: the forward stores the library's
recording id, and a backward whose recording has been replaced or extended
since then raises instead of returning another run's gradients.
"""
import torch

from . import binding as pm


class StaleRecordingError(RuntimeError):
    """The library context no longer holds the forward this backward belongs to."""


class PmRun(torch.autograd.Function):
    """u_0(T) as a function of the cell-centred sigma_a and sigma_s.

    spec: dict with keys N, dx, dt, nsteps, checkpoint (k > 0), moments
    (callable i -> [nz, ny, nx] float64 initial plane), optional q and
    precision (binding.PM_FP64 or PM_FP32).
    """

    @staticmethod
    def forward(ctx, sigma_a, sigma_s, spec):
        shape = tuple(sigma_a.shape)
        nz, ny, nx = shape
        dev = sigma_a.device if sigma_a.is_cuda else torch.device("cuda", 0)
        sa = sigma_a.detach().to("cpu", torch.float64).numpy()
        ss = sigma_s.detach().to("cpu", torch.float64).numpy()
        pm.pm_set_precision(spec.get("precision", pm.PM_FP64))
        pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
        pm.pm_init(spec["N"], nx, ny, nz, spec["dx"], spec["dt"], sa, ss, spec.get("q"))
        V = (spec["N"] + 1) ** 2
        for i in range(V):
            pm.pm_write(i, spec["moments"](i))
        pm.pm_set_checkpoint(int(spec.get("checkpoint", 20)))
        pm.pm_step(int(spec["nsteps"]))
        out = torch.empty(shape, dtype=torch.float64, device=dev)
        pm.pm_read_dev(0, out.data_ptr())
        ctx.shape = shape
        ctx.dev = dev
        ctx.in_dev = sigma_a.device
        ctx.recording = pm.pm_recording_id()
        return out

    @staticmethod
    def backward(ctx, grad_u0):
        if pm.pm_recording_id() != ctx.recording:
            raise StaleRecordingError(
                "libpm's recorded forward changed since this forward ran (another forward, "
                "pm_init, pm_write, pm_step or pm_finalize came in between); run each "
                "backward before the next forward")
        g = grad_u0.detach().to(ctx.dev, torch.float64).contiguous()
        dsa = torch.empty(ctx.shape, dtype=torch.float64, device=ctx.dev)
        dss = torch.empty(ctx.shape, dtype=torch.float64, device=ctx.dev)
        pm.pm_bind_stream(torch.cuda.current_stream(ctx.dev).cuda_stream)
        pm.pm_grad_dev(g.data_ptr(), dsa.data_ptr(), dss.data_ptr())
        return dsa.to(ctx.in_dev), dss.to(ctx.in_dev), None


def run_u0(sigma_a, sigma_s, spec):
    return PmRun.apply(sigma_a, sigma_s, spec)
