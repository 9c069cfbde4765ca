"""PyTorch convenience layer over the C ABI: device tensors in, device tensors
out.  PyTorch provides device memory and streams only; every step of the
matrix-element evaluation runs in the HIP kernels behind ``binding``."""
from __future__ import annotations

import torch

from . import binding as B

PROCESS_NAMES = {
    "eemumu": "e+ e- > mu+ mu-",
    "ggtt": "g g > t t~",
    "ggttg": "g g > t t~ g",
    "ggttgg": "g g > t t~ g g",
    "ggttggg": "g g > t t~ g g g",
    "uutt": "u u~ > t t~",
    "uxutt": "u~ u > t t~",
    "uuttg": "u u~ > t t~ g",
    "uxuttg": "u~ u > t t~ g",
    "ugttu": "u g > t t~ u",
    "guttu": "g u > t t~ u",
    "uxgttux": "u~ g > t t~ u~",
    "guxttux": "g u~ > t t~ u~",
    "uuttgg": "u u~ > t t~ g g",
    "uxuttgg": "u~ u > t t~ g g",
    "ugttug": "u g > t t~ u g",
    "guttug": "g u > t t~ u g",
    "uxgttuxg": "u~ g > t t~ u~ g",
    "guxttuxg": "g u~ > t t~ u~ g",
    "ggttuux": "g g > t t~ u u~",
    "uuttuux": "u u~ > t t~ u u~",
    "uuttddx": "u u~ > t t~ d d~",
    "uuttuu": "u u > t t~ u u",
    "udttud": "u d > t t~ u d",
    "uxuxttuxux": "u~ u~ > t t~ u~ u~",
}


class ChannelMix:
    """Several subprocesses of one final state behind one call: event e is
    evaluated by channel[e] (an index into `processes`), optionally at its own
    alpha_s."""

    def __init__(self, processes, precision: str = "fp64", filter_helicities: bool = True, noalloc: bool = False,
                 **params):
        self.members = [MatrixElement(p, precision, filter_helicities, **params) for p in processes]
        # noalloc: the entry point whose workspace is the library's fixed
        # device array (for callers that cannot allocate)
        self.call = B.me_compute_channels_noalloc if noalloc else B.me_compute_channels

    def __call__(self, momenta: torch.Tensor, channel: torch.Tensor, alphas: torch.Tensor | None = None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        npar = self.members[0].info["npar"]
        if momenta.dtype != torch.float64 or not momenta.is_cuda or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 CUDA tensor [nevt][npar][4]")
        if momenta.dim() != 3 or momenta.shape[1] != npar or momenta.shape[2] != 4:
            raise ValueError(f"momenta must have shape [nevt][{npar}][4]")
        n = momenta.shape[0]
        if channel.shape != (n,) or not channel.is_cuda or channel.device != momenta.device:
            raise ValueError("channel must be a CUDA tensor of nevt integers on the momenta's device")
        if alphas is not None and (alphas.shape != (n,) or not alphas.is_cuda or alphas.device != momenta.device):
            raise ValueError("alphas must be a CUDA tensor of nevt values on the momenta's device")
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        elif out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
            raise ValueError("out must be a contiguous float64 CUDA tensor with nevt elements")
        ch = channel.to(dtype=torch.int32).contiguous()
        a = alphas.to(dtype=torch.float64).contiguous() if alphas is not None else None
        self.call([m.handle for m in self.members], momenta.data_ptr(), ch.data_ptr(),
                  a.data_ptr() if a is not None else 0, n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return out

    def close(self):
        for m in self.members:
            m.close()


class MatrixElement:
    """One process handle.  precision: "fp64", "mixed" (colour sum on the
    unit measured fastest for the process), "mixed_mfma16" (FP16 hi+lo MFMA),
    "mixed_mfma32" (FP32 MFMA), "mixed_mfma_bf16" (BF16 hi+lo MFMA) or
    "mixed_valu" (vector ALU)."""

    def __init__(self, process: str, precision: str = "fp64", filter_helicities: bool = True, **params):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the matrix-element engine has no CPU path")
        prm = B.me_default_params(**params)
        prm.precision = {"fp64": B.ME_FP64, "mixed": B.ME_MIXED, "mixed_valu": B.ME_MIXED_VALU,
                         "mixed_mfma32": B.ME_MIXED_MFMA32, "mixed_mfma16": B.ME_MIXED_MFMA16,
                         "mixed_mfma_bf16": B.ME_MIXED_MFMABF16}[precision]
        self.process = PROCESS_NAMES.get(process, process)
        self.handle = B.me_create(self.process, prm)
        if filter_helicities:
            B.me_helicity_filter(self.handle)
        self.info = B.me_info(self.handle)

    def __call__(self, momenta: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if momenta.dtype != torch.float64 or not momenta.is_cuda or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 CUDA tensor [nevt][npar][4]")
        if momenta.dim() != 3 or momenta.shape[1] != self.info["npar"] or momenta.shape[2] != 4:
            raise ValueError(f"momenta must have shape [nevt][{self.info['npar']}][4]")
        n = momenta.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        elif out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
            raise ValueError("out must be a contiguous float64 CUDA tensor with nevt elements")
        B.me_compute(self.handle, momenta.data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return out

    def helicities(self, momenta: torch.Tensor) -> torch.Tensor:
        if momenta.dtype != torch.float64 or not momenta.is_cuda or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 CUDA tensor [nevt][npar][4]")
        if momenta.dim() != 3 or momenta.shape[1] != self.info["npar"] or momenta.shape[2] != 4:
            raise ValueError(f"momenta must have shape [nevt][{self.info['npar']}][4]")
        n = momenta.shape[0]
        out = torch.empty((n, self.info["nhel"]), dtype=torch.float64, device=momenta.device)
        B.me_compute_helicities(self.handle, momenta.data_ptr(), n, out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
        return out

    def good_helicities(self):
        return B.me_good_helicities(self.handle)

    def close(self):
        if self.handle:
            B.me_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
