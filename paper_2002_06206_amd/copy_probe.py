"""Counter calibration: runs the library's plain FP64 copy kernel (ibm_get_rhs,
N doubles read and N doubles written) a few times at 256^3 so that rocprofv3
FETCH_SIZE / WRITE_SIZE can be scaled against a kernel of known traffic."""
import torch

from paper_2002_06206_amd import ibm


def main(n=256, reps=5):
    torch.cuda.set_device(0)
    s = ibm.Solver((n, n, n), 1.0, (0.0, 0.0, 0.0), (ibm.INFLOW, ibm.OUTFLOW) + (ibm.SLIP,) * 4, (1.0, 0.0, 0.0))
    blocked = torch.zeros((n, n, n), dtype=torch.uint8, device="cuda")
    theta = torch.full((n, n, n, 6), 2.0, dtype=torch.float64, device="cuda")
    s.build(blocked, theta)
    out = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    for _ in range(reps):
        ibm.ibm_get_rhs(s.ctx, out)
    torch.cuda.synchronize()
    print("copy probe: %d x %d doubles read and written" % (reps, n ** 3))


if __name__ == "__main__":
    main()
