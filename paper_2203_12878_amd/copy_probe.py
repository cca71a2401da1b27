"""A plain device copy of known size, used to calibrate the HBM byte
counters (FETCH_SIZE / WRITE_SIZE) that measure the kernels' traffic:
bytes counted for this copy vs. the bytes it must move give the factor
applied to the kernels' counter readings.

    python -m paper_2203_12878_amd.copy_probe [MiB]
"""
import sys


def main():
    import torch
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d bytes (read %d, write %d)" % (n, n, n), flush=True)


if __name__ == "__main__":
    main()
