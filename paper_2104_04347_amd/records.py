"""Keys of the committed per-kernel records under profiles/ (traffic.json,
valu_insts.json, clock.json): one name per kernel build and launch, shared by
the benchmark, which reads the records, and the tools that write them."""
from __future__ import annotations


def key_1d(precision: str, P: int, variant: int) -> tuple:
    """Key and kernel source set of the 1D Euler half-step kernel (limiter on)
    in launch variant `variant`."""
    bulk = "f64" if precision == "fp64" else "f32"
    if variant == 4:
        return f"k_half_step_wide<euler,P={P},limiter,{bulk}>", "1d_wide"
    return f"k_half_step<euler,P={P},limiter,{bulk},variant={variant}>", "1d"


ROWS_FORM = {1: "no prefetch", 2: "prefetch", 3: "prefetch,bands"}


def kernel_2d(equation: str, P: int, limiter: bool, variant: int) -> str:
    form = ROWS_FORM.get(variant, "8x8 tiles")
    return f"k2d_half_step_rows<{equation},P={P},{'limiter' if limiter else 'no limiter'},{form}>"


def key_2d(equation: str, P: int, limiter: bool, variant: int, periodic: bool, threads: int, blocks: int) -> str:
    """Key of the 2D half-step kernel: the kernel, the edges and the launch
    grid actually run (the grid sets how many priming rows are re-read)."""
    return (kernel_2d(equation, P, limiter, variant) + ("" if periodic else ",transmissive") +
            f",grid={threads}x{blocks}")
