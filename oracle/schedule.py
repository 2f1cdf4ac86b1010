"""O8: the block schedule that enriches the plan Pi, and its SELL-C-sigma
storage (test infrastructure only, like the rest of this package).

Section "PSGE: panel-structured Gaussian elimination" ("Why Pi must be
enriched") asks symbolic preprocessing to emit, besides the CSR arrays, panel
boundaries (contiguous column segments in dictionary order) and the
row-to-panel incidence; section "Row assembly as a dictionary join;
divergence control via SELL-C-sigma bucketing" buckets rows by length,
sorting locally within windows and padding inside fixed-size slices.  The
paper fixes neither the panel widths nor how windows and slices meet panels;
the readings taken here:

* Panels: P_l = columns [l W, (l + 1) W) for a width W; a row belongs to the
  panel of its leading (first) column; empty rows form a last group after
  the panels.
* Within each panel, rows in increasing row index are cut into windows of
  sigma consecutive rows; each window is sorted by length, longest first,
  ties by row index.
* Slices: consecutive runs of C rows of a panel's sorted list (the last one
  of a panel may be shorter; no slice spans two panels); a slice's width is
  its longest row.
* SELL storage: slice s occupies C * width_s slots from its offset (an
  exclusive scan of C * width); the k-th entry of the slice's j-th row is at
  offset + k C + j; padding has column 0 and value 0.

Everything is plain Python lists and sorts.
"""


def block_schedule(row_ptr, col_ind, N, W, C, sigma):
    """The schedule of a CSR matrix with N columns: perm (rows in schedule
    order), panel_ptr (npanels + 2 offsets into perm: the panels, then the
    empty rows), slice_start (offsets into perm), slice_panel, slice_width,
    slice_off (npslices + 1 offsets into the SELL storage)."""
    r = len(row_ptr) - 1
    npanels = max(1, -(-N // W))
    length = [row_ptr[i + 1] - row_ptr[i] for i in range(r)]
    panel = [col_ind[row_ptr[i]] // W if length[i] else npanels for i in range(r)]
    perm, panel_ptr = [], [0]
    for l in range(npanels + 1):
        rows = [i for i in range(r) if panel[i] == l]
        for w0 in range(0, len(rows), sigma):
            win = rows[w0:w0 + sigma]
            perm += sorted(win, key=lambda i: (-length[i], i))
        panel_ptr.append(len(perm))
    slice_start, slice_panel, slice_width, slice_off = [], [], [], [0]
    for l in range(npanels + 1):
        for s0 in range(panel_ptr[l], panel_ptr[l + 1], C):
            rows = perm[s0:min(s0 + C, panel_ptr[l + 1])]
            slice_start.append(s0)
            slice_panel.append(l)
            slice_width.append(max(length[i] for i in rows))
            slice_off.append(slice_off[-1] + C * slice_width[-1])
    return {"perm": perm, "panel_ptr": panel_ptr, "slice_start": slice_start, "slice_panel": slice_panel,
            "slice_width": slice_width, "slice_off": slice_off, "npanels": npanels}


def sell_storage(row_ptr, col_ind, val, sched, C):
    """The padded column-major slices: (cols, vals) of length slice_off[-1]."""
    total = sched["slice_off"][-1]
    cols, vals = [0] * total, [0] * total
    ends = sched["slice_start"][1:] + [len(sched["perm"])]
    for s, s0 in enumerate(sched["slice_start"]):
        s1 = min(s0 + C, sched["panel_ptr"][sched["slice_panel"][s] + 1], ends[s])
        for j, i in enumerate(sched["perm"][s0:s1]):
            for k, e in enumerate(range(row_ptr[i], row_ptr[i + 1])):
                at = sched["slice_off"][s] + k * C + j
                cols[at] = col_ind[e]
                vals[at] = val[e]
    return cols, vals
