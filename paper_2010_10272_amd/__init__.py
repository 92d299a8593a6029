"""MI355X-native km1 label-propagation refinement core (arXiv 2010.10272).

The compute path is the HIP library ``libhgref.so`` behind the C ABI in
``include/hgref.h``; ``paper_2010_10272_amd.hgref`` is its Python binding.
The binding is imported on first use so that ``python -m
paper_2010_10272_amd.build`` works before the library exists.
"""


def __getattr__(name):
    if name == "hgref":
        import importlib
        return importlib.import_module(".hgref", __name__)
    raise AttributeError(name)
