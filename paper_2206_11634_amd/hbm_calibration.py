"""Reference kernel for scaling HBM traffic counters.

    python -m paper_2206_11634_amd.hbm_calibration

runs one elementwise kernel (out = in * 1) over 19 planes of 512^3 floats:
10.201 GB read and 10.201 GB written per dispatch.  Under
`rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) the counter values of that
dispatch give the factor between the counters' units and bytes on this
device, which converts the counters of the lattice kernels to bytes."""
import torch

N = 19 * 512 ** 3


def main(reps: int = 3):
    a = torch.zeros(N, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(f"elementwise copy: {N * 4 / 1e9:.3f} GB read and written per dispatch, {reps} dispatches")


if __name__ == "__main__":
    main()
