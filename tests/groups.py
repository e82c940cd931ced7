"""Which signals share a checksum group in one call (test helper).

Directly addressed launches form G groups (G = workgroups x sub-signals per
workgroup for a single pass, one per group of tiles for a two-pass chunk);
transaction b of group g transforms signal g + b G (include/tfft.h,
tfft_route_info).  `info` is paper_2412_05824_amd.route_info() of the length;
`batch` the signals of the call (of the chunk, for two passes)."""


def group_of(sig: int, batch: int, info: dict) -> list:
    T = info["T"]
    if info["passes"] == 1:
        s = info["slots0"]
        groups = -(-batch // (s * T)) * s
    else:
        groups = -(-batch // T)
    g = sig % groups
    return [g + b * groups for b in range(T) if g + b * groups < batch]
